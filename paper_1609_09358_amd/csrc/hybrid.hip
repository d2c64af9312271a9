// hybrid.hip -- hybrid BP -> CA-SCL decoder (Sec. III, Fig. 3).
//
// The CPU scheduling loop of Fig. 3 becomes four kernels on one stream with
// no host round trip: BP on every frame, compaction of the frames whose BP
// verdict is not ok into a device queue ("copy failed CWs to buffer"),
// persistent CA-SCL workgroups that read the queue length on the device, and
// a merge that emits the information bits and statistics.
#include "internal.hpp"

namespace polarhip {
namespace {

__global__ void clear_count_kernel(int32_t* count) {
    if (threadIdx.x == 0) *count = 0;
}

// queue[] <- ids of frames with ok == 0; one atomic per wavefront
__global__ __launch_bounds__(256) void compact_kernel(const uint8_t* __restrict__ ok, int64_t B,
                                                      int32_t* __restrict__ queue, int32_t* __restrict__ count) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool fail = f < B && ok[f] == 0;
    const uint64_t m = __ballot(fail);
    const int lane = __lane_id();
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(count, (int)__popcll(m));
    base = __shfl(base, 0, 64);
    if (fail) queue[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)f;
}

// info_hat <- information bits of u_hat (BP result or its SCL replacement);
// 32 frames per workgroup, statistics reduced per wavefront before the atomics
constexpr int kMergeFrames = 32;

__global__ __launch_bounds__(256) void merge_kernel(CodeDev code, const uint8_t* __restrict__ u_hat,
                                                    const uint8_t* __restrict__ ok,
                                                    const int32_t* __restrict__ iters,
                                                    const uint8_t* __restrict__ scl_ok, int64_t B,
                                                    uint8_t* __restrict__ info_hat, uint8_t* __restrict__ used_scl,
                                                    unsigned long long* __restrict__ stats) {
    const int K = code.K, N = code.N;
    const int64_t f0 = (int64_t)blockIdx.x * kMergeFrames;
    const int nf = (int)((B - f0) < kMergeFrames ? (B - f0) : kMergeFrames);
    for (int it = threadIdx.x; it < nf * K; it += blockDim.x) {
        const int lf = it / K, q = it - lf * K;
        const int64_t f = f0 + lf;
        info_hat[f * K + q] = u_hat[f * N + code.info_pos[q]];
    }
    if (threadIdx.x < 64) {
        const int lf = threadIdx.x;
        unsigned long long s_bp = 0, s_scl = 0, s_it = 0, s_fail = 0, s_n = 0;
        if (lf < nf) {
            const int64_t f = f0 + lf;
            const bool good = ok[f] != 0;
            if (used_scl) used_scl[f] = good ? 0 : 1;
            s_n = 1;
            s_bp = good;
            s_scl = !good;
            s_it = (unsigned long long)iters[f];
            s_fail = (!good && !scl_ok[f]) ? 1ull : 0ull;
        }
        if (stats) {
            for (int m = 32; m >= 1; m >>= 1) {
                s_n += __shfl_xor(s_n, m, 64);
                s_bp += __shfl_xor(s_bp, m, 64);
                s_scl += __shfl_xor(s_scl, m, 64);
                s_it += __shfl_xor(s_it, m, 64);
                s_fail += __shfl_xor(s_fail, m, 64);
            }
            if (lf == 0) {
                atomicAdd(&stats[0], s_n);
                if (s_bp) atomicAdd(&stats[1], s_bp);
                if (s_scl) atomicAdd(&stats[2], s_scl);
                atomicAdd(&stats[3], s_it);
                if (s_fail) atomicAdd(&stats[4], s_fail);
            }
        }
    }
}

struct HybridWs {
    uint8_t* u_hat;
    uint8_t* ok;
    int32_t* iters;
    int32_t* queue;
    int32_t* count;
    uint8_t* scl_ok;
    void* scl_glob;
    size_t total;
};

HybridWs carve(const polar_code* code, int64_t B, const SclPlan& plan, void* base) {
    HybridWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_u = take((size_t)B * code->N);
    const size_t o_ok = take((size_t)B);
    const size_t o_it = take((size_t)B * 4);
    const size_t o_q = take((size_t)B * 4);
    const size_t o_c = take(4);
    const size_t o_s = take((size_t)B);
    const size_t o_g = take(plan.glob_per_wg * plan.grid);
    w.total = off;
    if (base) {
        char* b = static_cast<char*>(base);
        w.u_hat = reinterpret_cast<uint8_t*>(b + o_u);
        w.ok = reinterpret_cast<uint8_t*>(b + o_ok);
        w.iters = reinterpret_cast<int32_t*>(b + o_it);
        w.queue = reinterpret_cast<int32_t*>(b + o_q);
        w.count = reinterpret_cast<int32_t*>(b + o_c);
        w.scl_ok = reinterpret_cast<uint8_t*>(b + o_s);
        w.scl_glob = plan.glob_per_wg ? (void*)(b + o_g) : nullptr;
    }
    return w;
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

static polar_status check_bp_params(const polar_code* code, const bp_params* p) {
    if (p->max_iter < 1) return set_error(POLAR_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (p->stop < 0 || p->stop > 2) return set_error(POLAR_ERR_INVALID_ARG, "stop must be 0, 1 or 2");
    if (p->stop == 2 && code->c == 0) return set_error(POLAR_ERR_INVALID_ARG, "CRC stop needs a code with a CRC");
    if (!(p->llr_max > 0.0f)) return set_error(POLAR_ERR_INVALID_ARG, "llr_max must be > 0");
    if (p->rule != 0) return set_error(POLAR_ERR_UNSUPPORTED, "only the min-sum rule runs on GPU");
    if (p->weights && p->weight_iters < p->max_iter) return set_error(POLAR_ERR_INVALID_ARG, "weight_iters < max_iter");
    if (p->variant != 0 && !bp_variant_supported(code->n, p->variant))
        return set_error(POLAR_ERR_INVALID_ARG, "unknown BP variant");
    return POLAR_OK;
}

extern "C" polar_status polar_workspace_size(const polar_code* code, int64_t B, int32_t L, const bp_params* params,
                                             size_t* bytes) {
    if (!code || !bytes || B < 0) return set_error(POLAR_ERR_INVALID_ARG, "polar_workspace_size: bad argument");
    SclPlan plan;
    polar_status st = scl_plan(code, L, B > 0 ? B : 1, &plan);
    if (st != POLAR_OK) return st;
    if (!params) {
        *bytes = plan.glob_per_wg * plan.grid;
    } else {
        *bytes = carve(code, B, plan, nullptr).total;
    }
    return ok_status();
}

extern "C" polar_status hybrid_decode_batch(const polar_code* code, const float* llr, int64_t B,
                                            const bp_params* p, int32_t L, uint8_t* info_hat, uint8_t* used_scl,
                                            int64_t* stats, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!code || !p) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch: null code or params");
    if (B < 0 || B > (int64_t)INT32_MAX) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch: bad batch size");
    if (B > 0 && (!llr || !info_hat)) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch: null buffer");
    polar_status st = check_bp_params(code, p);
    if (st != POLAR_OK) return st;
    SclPlan plan;
    if ((st = scl_plan(code, L, B > 0 ? B : 1, &plan)) != POLAR_OK) return st;
    HybridWs w = carve(code, B, plan, nullptr);
    if (!ws || ws_bytes < w.total) return set_error(POLAR_ERR_WORKSPACE, "hybrid_decode_batch: workspace too small");
    if (B == 0) return ok_status();
    w = carve(code, B, plan, ws);
    if ((st = launch_bp(code, llr, B, p, w.u_hat, nullptr, w.iters, w.ok, stream)) != POLAR_OK) return st;
    hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(64), 0, stream, w.count);
    const unsigned cblocks = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(compact_kernel, dim3(cblocks), dim3(256), 0, stream, w.ok, B, w.queue, w.count);
    if ((st = hip_check(hipGetLastError(), "compact launch")) != POLAR_OK) return st;
    if ((st = launch_scl(code, plan, llr, L, w.queue, w.count, 0, w.u_hat, w.scl_ok, nullptr, w.scl_glob, stream)) !=
        POLAR_OK)
        return st;
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((B + kMergeFrames - 1) / kMergeFrames)), dim3(256), 0, stream, code->dev(), w.u_hat, w.ok, w.iters,
                       w.scl_ok, B, info_hat, used_scl, reinterpret_cast<unsigned long long*>(stats));
    if ((st = hip_check(hipGetLastError(), "merge launch")) != POLAR_OK) return st;
    return ok_status();
}
