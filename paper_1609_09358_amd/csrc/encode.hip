// encode.hip -- polar encoder x = u G (Sec. II, Fig. 1) and the BPSK/AWGN
// channel used to synthesise workloads.
#include "internal.hpp"

namespace polarhip {
namespace {

constexpr int ENC_THREADS = 256;

// One workgroup per frame.  u is assembled in LDS (info bits, then the CRC
// obtained by linearity from the per-bit CRC table), then the n butterfly
// stages of Fig. 1 run in place: at distance d, u[i] ^= u[i + d] for i & d == 0.
__global__ __launch_bounds__(ENC_THREADS) void encode_kernel(CodeDev code, const uint8_t* __restrict__ info,
                                                             uint8_t* __restrict__ u_out,
                                                             uint8_t* __restrict__ x_out) {
    extern __shared__ uint8_t su[];
    __shared__ uint32_t red[ENC_THREADS / 64];
    const int N = code.N, K = code.K, c = code.c;
    const int64_t f = gid_x();
    const uint8_t* in = info + f * K;
    for (int i = lid_x(); i < N; i += ENC_THREADS) su[i] = 0;
    __syncthreads();
    uint32_t crc = 0;
    for (int q = lid_x(); q < K; q += ENC_THREADS) {
        uint8_t b = in[q] & 1u;
        su[code.info_pos[q]] = b;
        if (b && c) crc ^= code.enc_crc[q];
    }
    if (c) {
        for (int m = 32; m >= 1; m >>= 1) crc ^= __shfl_xor(crc, m);
        if ((lid_x() & 63) == 0) red[lid_x() >> 6] = crc;
    }
    __syncthreads();
    if (c) {
        crc = 0;
        for (int w = 0; w < ENC_THREADS / 64; ++w) crc ^= red[w];
        for (int j = lid_x(); j < c; j += ENC_THREADS) su[code.info_pos[K + j]] = (crc >> (c - 1 - j)) & 1u;
    }
    __syncthreads();
    if (u_out)
        for (int i = lid_x(); i < N; i += ENC_THREADS) u_out[f * N + i] = su[i];
    __syncthreads();
    for (int d = 1; d < N; d <<= 1) {
        for (int p = lid_x(); p < N / 2; p += ENC_THREADS) {
            int i = (p / d) * 2 * d + (p % d);
            su[i] ^= su[i + d];
        }
        __syncthreads();
    }
    for (int i = lid_x(); i < N; i += ENC_THREADS) x_out[f * N + i] = su[i];
}

__global__ void channel_kernel(const uint8_t* __restrict__ x, const float* __restrict__ z,
                               const float* __restrict__ sigma2, int64_t total, int32_t N,
                               float* __restrict__ llr) {
    int64_t idx = gid_x() * wg_size_x() + lid_x();
    if (idx >= total) return;
    float s2 = sigma2[idx / N];
    float y = (x[idx] ? -1.0f : 1.0f) + sqrtf(s2) * z[idx];
    llr[idx] = 2.0f * y / s2;
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

extern "C" polar_status polar_encode(const polar_code* code, const uint8_t* info, int64_t B,
                                     uint8_t* u_out, uint8_t* x_out, hipStream_t stream) {
    if (!code || !x_out || (B > 0 && !info)) return set_error(POLAR_ERR_INVALID_ARG, "polar_encode: null argument");
    if (B < 0 || B > (int64_t)INT32_MAX) return set_error(POLAR_ERR_INVALID_ARG, "polar_encode: bad batch size");
    if (B == 0) return ok_status();
    hipLaunchKernelGGL(encode_kernel, dim3((unsigned)B), dim3(ENC_THREADS), code->N, stream, code->dev(), info,
                       u_out, x_out);
    return hip_check(hipGetLastError(), "encode_kernel launch") == POLAR_OK ? ok_status() : POLAR_ERR_DEVICE;
}

extern "C" polar_status polar_channel_awgn(const uint8_t* x, const float* z, const float* sigma2, int64_t B,
                                           int32_t N, float* llr, hipStream_t stream) {
    if (!x || !z || !sigma2 || !llr) return set_error(POLAR_ERR_INVALID_ARG, "polar_channel_awgn: null argument");
    if (B < 0 || N <= 0) return set_error(POLAR_ERR_INVALID_ARG, "polar_channel_awgn: bad sizes");
    int64_t total = B * (int64_t)N;
    if (total == 0) return ok_status();
    unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(channel_kernel, dim3(blocks), dim3(256), 0, stream, x, z, sigma2, total, N, llr);
    return hip_check(hipGetLastError(), "channel_kernel launch") == POLAR_OK ? ok_status() : POLAR_ERR_DEVICE;
}
