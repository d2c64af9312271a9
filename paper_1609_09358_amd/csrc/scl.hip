// scl.hip -- CRC-aided successive-cancellation list decoder (Sec. II-A).
//
// One wavefront decodes one frame at a time; workgroups stay resident and walk
// a list of frames (a device-side count, so the hybrid decoder can feed it the
// compacted BP failures without a host round trip).
//
// Per path slot the wavefront keeps the LLR tree (level d holds 2^d values,
// level n is the channel) and the partial sums.  Paths are copied lazily: each
// slot keeps, per level, the slot whose array it reads.  Bit i rewrites
// levels ctz(i)..0 of every path into the path's own slot and reads level
// ctz(i)+1 through the pointer, which no path writes during bit i; partial
// sums are handled the same way.  A branching path therefore copies only its
// pointer vector.  Survivors are chosen by rank among the 2L candidates under
// the order (metric, parent list position, bit) -- the pruned pseudo sort of
// Sec. II-A with a strict tie rule -- and a survivor's new slot is its rank,
// so slot index and list position coincide.  The CRC is tracked per path as a
// running syndrome (linear in the decided bits); the decoded bits of the
// chosen path are recovered from a per-information-bit trace of
// (parent, bit).  Small levels live in LDS; the largest levels can be placed
// in a per-workgroup global slice to raise the number of resident frames.
#include "internal.hpp"

namespace polarhip {
namespace scl {

__device__ __forceinline__ float g_ms(float a, float b) {
    float m = fminf(fabsf(a), fabsf(b));
    uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(m) | s);
}

__device__ __forceinline__ void wave_mem_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wg_mem_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct Layout {
    int gl;   // levels < gl in LDS
    int sl;   // LDS stride of one slot's LLR levels (floats)
    int psl;  // LDS stride of one slot's partial sums (bytes)
};

template <int L>
__global__ __launch_bounds__(64) void scl_kernel(CodeDev code, const float* __restrict__ llr,
                                                 const int32_t* __restrict__ frame_ids,
                                                 const int32_t* __restrict__ count_dev, int64_t count_host,
                                                 uint8_t* __restrict__ u_hat, uint8_t* __restrict__ crc_ok,
                                                 float* __restrict__ pm_out, float* __restrict__ glam_all,
                                                 uint8_t* __restrict__ gps_all, Layout lay) {
    extern __shared__ __attribute__((aligned(16))) unsigned char sm[];
    const int lane = threadIdx.x;
    const int n = code.n, N = code.N, k = code.k;
    const int gl = lay.gl, SL = lay.sl, PSL = lay.psl;

    float* slam = reinterpret_cast<float*>(sm);                                  // [L][SL]
    float* scr_pm = slam + L * SL;                                               // [L]
    uint32_t* scr_syn = reinterpret_cast<uint32_t*>(scr_pm + L);                 // [L]
    uint8_t* sps = reinterpret_cast<uint8_t*>(scr_syn + L);                      // [L][PSL]
    uint8_t* ptrA = sps + L * PSL;                                               // [2][L][16] LLR level pointers
    uint8_t* ptrB = ptrA + 2 * L * 16;                                           // [2][L][16] partial-sum pointers
    uint8_t* scr_par = ptrB + 2 * L * 16;                                        // [L]
    uint8_t* scr_bit = scr_par + L;                                              // [L]
    uint8_t* dec = scr_bit + L;                                                  // [N]
    uint8_t* tbk = dec + N;                                                      // [k][L]

    float* glam = glam_all ? glam_all + (size_t)blockIdx.x * L * N : nullptr;
    uint8_t* gps = gps_all ? gps_all + (size_t)blockIdx.x * L * N : nullptr;

    auto lam_rd = [&](int slot, int d, int e) -> float {
        return d < gl ? slam[slot * SL + (1 << d) + e] : glam[(size_t)slot * N + (1 << d) + e];
    };
    auto lam_wr = [&](int slot, int d, int e, float v) {
        if (d < gl) slam[slot * SL + (1 << d) + e] = v;
        else glam[(size_t)slot * N + (1 << d) + e] = v;
    };
    auto ps_rd = [&](int slot, int d, int e) -> uint8_t {
        return d < gl ? sps[slot * PSL + (1 << d) + e] : gps[(size_t)slot * N + (1 << d) + e];
    };
    auto ps_wr = [&](int slot, int d, int e, uint8_t v) {
        if (d < gl) sps[slot * PSL + (1 << d) + e] = v;
        else gps[(size_t)slot * N + (1 << d) + e] = v;
    };
    auto order = [&](int d) {
        if (d < gl) wave_mem_order(); else wg_mem_order();
    };

    const int64_t count = count_dev ? (int64_t)(*count_dev) : count_host;
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
        const int64_t f = frame_ids ? (int64_t)frame_ids[q] : q;
        const float* chan = llr + f * N;

        // initial list: one path in slot 0, all pointers to slot 0
        for (int it = lane; it < 2 * 2 * L * 16; it += 64) ptrA[it] = 0;  // ptrA and ptrB are contiguous
        for (int it = lane; it < N; it += 64) dec[it] = 0;
        int act = 1;
        int cur = 0;
        float PM = 0.0f;
        uint32_t SYN = 0u;
        int infoq = 0;
        wave_mem_order();

        for (int i = 0; i < N; ++i) {
            const int top = (i == 0) ? n - 1 : __builtin_ctz((unsigned)i);
            float lam_own = 0.0f;
            // ---- LLR levels top..0
            for (int d = top; d >= 0; --d) {
                const int sz = 1 << d;
                const int items = act << d;
                for (int it = lane; it < items; it += 64) {
                    const int slot = it >> d;
                    const int e = it & (sz - 1);
                    float a, b;
                    if (d + 1 == n) {
                        a = chan[e];
                        b = chan[e + sz];
                    } else {
                        const int src = (d == top) ? ptrA[(cur * L + slot) * 16 + d + 1] : slot;
                        a = lam_rd(src, d + 1, e);
                        b = lam_rd(src, d + 1, e + sz);
                    }
                    float val;
                    if (d == top && i != 0) {
                        const int ps_src = ptrB[(cur * L + slot) * 16 + d];
                        val = ps_rd(ps_src, d, e) ? b - a : b + a;
                    } else {
                        val = g_ms(a, b);
                    }
                    lam_wr(slot, d, e, val);
                    if (d == 0) lam_own = val;
                }
                order(d);
            }
            // levels 0..top are now owned by every path
            for (int it = lane; it < act * (top + 1); it += 64) {
                const int slot = it / (top + 1), d = it % (top + 1);
                ptrA[(cur * L + slot) * 16 + d] = (uint8_t)slot;
            }
            // ---- decision
            int bit = 0;
            const bool frozen = (code.frozen_bits[i >> 5] >> (i & 31)) & 1u;
            if (frozen) {
                if (lane < act) {
                    const float pen = lam_own < 0.0f ? fabsf(lam_own) : 0.0f;
                    PM = PM + pen;
                }
            } else {
                const int ncand = 2 * act;
                const int p = lane >> 1, b = lane & 1;
                const float lp = __shfl(lam_own, p, 64);
                const float pmp = __shfl(PM, p, 64);
                const uint32_t sp = __shfl(SYN, p, 64);
                const bool hd = lp < 0.0f;
                const float pen = (b != (int)hd) ? fabsf(lp) : 0.0f;
                const float met = pmp + pen;
                int rank = 0;
                for (int c2 = 0; c2 < ncand; ++c2) {
                    const float m2 = __shfl(met, c2, 64);
                    rank += (m2 < met || (m2 == met && c2 < lane)) ? 1 : 0;
                }
                const int nact = ncand < L ? ncand : L;
                const uint32_t syn_i = code.syn[i];
                if (lane < ncand && rank < L) {
                    scr_pm[rank] = met;
                    scr_syn[rank] = sp ^ (b ? syn_i : 0u);
                    scr_par[rank] = (uint8_t)p;
                    scr_bit[rank] = (uint8_t)b;
                }
                wave_mem_order();
                int par = 0;
                if (lane < nact) {
                    PM = scr_pm[lane];
                    SYN = scr_syn[lane];
                    par = scr_par[lane];
                    bit = scr_bit[lane];
                    tbk[infoq * L + lane] = (uint8_t)(par | (bit << 7));
                }
                const int nxt = cur ^ 1;
                for (int it = lane; it < nact * 16; it += 64) {
                    const int slot = it >> 4, d = it & 15;
                    const int ps = scr_par[slot];
                    ptrA[(nxt * L + slot) * 16 + d] = ptrA[(cur * L + ps) * 16 + d];
                    ptrB[(nxt * L + slot) * 16 + d] = ptrB[(cur * L + ps) * 16 + d];
                }
                wave_mem_order();
                cur = nxt;
                act = nact;
                ++infoq;
            }
            // ---- partial sums: finished sub-block of size 2^t goes to level t
            const int t = __builtin_ctz(~(unsigned)i);
            if (t < n) {
                const int base = (1 << t);
                if (lane < act) ps_wr(lane, t, base - 1, (uint8_t)bit);
                order(t);
                for (int d = 0; d < t; ++d) {
                    const int sz = 1 << d;
                    const int items = act << d;
                    for (int it = lane; it < items; it += 64) {
                        const int slot = it >> d, e = it & (sz - 1);
                        const int src = ptrB[(cur * L + slot) * 16 + d];
                        const uint8_t v = ps_rd(src, d, e) ^ ps_rd(slot, t, base - sz + e);
                        ps_wr(slot, t, base - 2 * sz + e, v);
                    }
                    order(t);
                }
                if (lane < act) ptrB[(cur * L + lane) * 16 + t] = (uint8_t)lane;
                wave_mem_order();
            }
        }
        // ---- selection: smallest (CRC fails, metric, position)
        uint64_t key = ~0ull;
        if (lane < act)
            key = ((uint64_t)(SYN != 0u) << 40) | ((uint64_t)__float_as_uint(PM) << 8) | (uint64_t)lane;
        for (int m = 32; m >= 1; m >>= 1) {
            const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)key, m, 64);
            key = o < key ? o : key;
        }
        const int best = (int)(key & 0xFF);
        const bool best_ok = ((key >> 40) & 1ull) == 0;
        const float best_pm = __shfl(PM, best, 64);
        // ---- trace back the chosen path through the information bits
        if (lane == 0) {
            int s = best;
            for (int qq = infoq - 1; qq >= 0; --qq) {
                const uint8_t e = tbk[qq * L + s];
                dec[code.info_pos[qq]] = e >> 7;
                s = e & 0x7F;
            }
        }
        wave_mem_order();
        for (int it = lane; it < N; it += 64) u_hat[f * N + it] = dec[it];
        if (lane == 0) {
            crc_ok[f] = best_ok ? 1 : 0;
            if (pm_out) pm_out[f] = best_pm;
        }
        wave_mem_order();
    }
}

using KernelFn = void (*)(CodeDev, const float*, const int32_t*, const int32_t*, int64_t, uint8_t*, uint8_t*,
                          float*, float*, uint8_t*, Layout);

KernelFn pick(int L) {
    switch (L) {
        case 1: return &scl_kernel<1>;
        case 2: return &scl_kernel<2>;
        case 4: return &scl_kernel<4>;
        case 8: return &scl_kernel<8>;
        case 16: return &scl_kernel<16>;
        case 32: return &scl_kernel<32>;
        default: return nullptr;
    }
}

size_t lds_bytes(int L, int N, int k, int gl) {
    const size_t sl = (size_t(1) << gl) + 1;
    const size_t psl = (size_t(1) << gl);
    size_t b = 0;
    b += (size_t)L * sl * 4;   // LLR levels
    b += (size_t)L * 4 * 2;    // scratch metric + syndrome
    b += (size_t)L * psl;      // partial sums
    b += (size_t)2 * L * 16 * 2;  // pointer vectors
    b += (size_t)L * 2;        // scratch parent + bit
    b += (size_t)N;            // decoded bits
    b += (size_t)k * L;        // trace
    return align_up(b, 16);
}

}  // namespace scl

static size_t g_scl_lds_budget = 48 * 1024;

polar_status scl_plan(const polar_code* code, int L, int64_t max_frames, SclPlan* plan) {
    scl::KernelFn fn = scl::pick(L);
    if (!fn) return set_error(POLAR_ERR_INVALID_ARG, "scl: L must be a power of two in [1, 32]");
    const int n = code->n, N = code->N, k = code->k;
    int gl = n;
    while (gl > 1 && scl::lds_bytes(L, N, k, gl) > g_scl_lds_budget) --gl;
    size_t lds = scl::lds_bytes(L, N, k, gl);
    if (lds > 160 * 1024) return set_error(POLAR_ERR_UNSUPPORTED, "scl: list too large for LDS");
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds);
    if (e != hipSuccess || per_cu <= 0) per_cu = 1;
    int64_t grid = (int64_t)device_cu_count() * per_cu;
    if (max_frames < grid) grid = max_frames;
    if (grid < 1) grid = 1;
    plan->gl = gl;
    plan->lds_bytes = lds;
    plan->glob_per_wg = (gl < n) ? (size_t)L * N * 5 : 0;
    plan->grid = (int)grid;
    return POLAR_OK;
}

polar_status launch_scl(const polar_code* code, const SclPlan& plan, const float* llr, int L,
                        const int32_t* frame_ids, const int32_t* count_dev, int64_t count_host, uint8_t* u_hat,
                        uint8_t* crc_ok, float* pm, void* glob, hipStream_t stream) {
    scl::KernelFn fn = scl::pick(L);
    float* glam = nullptr;
    uint8_t* gps = nullptr;
    if (plan.glob_per_wg) {
        glam = reinterpret_cast<float*>(glob);
        gps = reinterpret_cast<uint8_t*>(glam + (size_t)plan.grid * L * code->N);
    }
    scl::Layout lay;
    lay.gl = plan.gl;
    lay.sl = (1 << plan.gl) + 1;
    lay.psl = 1 << plan.gl;
    hipLaunchKernelGGL(fn, dim3(plan.grid), dim3(64), plan.lds_bytes, stream, code->dev(), llr, frame_ids,
                       count_dev, count_host, u_hat, crc_ok, pm, glam, gps, lay);
    return hip_check(hipGetLastError(), "scl_kernel launch");
}

}  // namespace polarhip

using namespace polarhip;

extern "C" polar_status scl_decode_batch(const polar_code* code, const float* llr, int64_t B, int32_t L,
                                         const int32_t* frame_ids, uint8_t* u_hat, uint8_t* crc_ok, float* pm,
                                         void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!code) return set_error(POLAR_ERR_INVALID_ARG, "scl_decode_batch: null code");
    if (B < 0) return set_error(POLAR_ERR_INVALID_ARG, "scl_decode_batch: negative batch");
    if (B > 0 && (!llr || !u_hat || !crc_ok)) return set_error(POLAR_ERR_INVALID_ARG, "scl_decode_batch: null buffer");
    SclPlan plan;
    polar_status st = scl_plan(code, L, B, &plan);
    if (st != POLAR_OK) return st;
    if (B == 0) return ok_status();
    const size_t need = plan.glob_per_wg * plan.grid;
    if (need && (!ws || ws_bytes < need)) return set_error(POLAR_ERR_WORKSPACE, "scl_decode_batch: workspace too small");
    st = launch_scl(code, plan, llr, L, frame_ids, nullptr, B, u_hat, crc_ok, pm, ws, stream);
    return st == POLAR_OK ? ok_status() : st;
}
