// wbp.hip -- weighted (learned) min-sum BP: loss, hand-written adjoint, weight
// gradient reduction and Adam.
//
// Forward: bp_kernel with weights and message saving (bp.hip): T iterations,
// no early stop, every produced row saved as saved[f][t][dir][s][node].
// Losses: binary cross-entropy of P(u_i = 1) = sigmoid(-lambda_i) over the
// non-frozen positions after the last iteration (or after every iteration),
// lambda = L_{i,1} + R_{i,1}; or the frame-failure surrogate, the probability
// (bits independent) that no iteration decides the whole frame right.
// Adjoint (reverse mode, by hand): iterations T..1; inside one, the L sweep is
// undone first (columns 0..n-1), then the R sweep (columns n-1..0), in the
// same register windows as the forward: adjoint rows cross window boundaries
// through the same LDS maps in the opposite direction.  Derivative rules:
// d clip(p)/dp = [|p| <= llr_max]; g(a,b) = a sgn(b) when |a| <= |b| (ties to
// a), else b sgn(a); the sign factor has zero derivative.  Every operation
// follows the CPU oracle's order, so a frame's gradient is bit-exact with the
// oracle's float build.  The per-frame weight gradient is written over the
// saved messages it no longer needs, and reduced over frames in frame order in
// double precision (deterministic).
#include "bp_common.hpp"

namespace polarhip {
namespace bp {

__device__ __forceinline__ void g_partials(float a, float b, float& da, float& db) {
    const float sb = (__float_as_uint(b) & 0x80000000u) ? -1.0f : 1.0f;
    const float sa = (__float_as_uint(a) & 0x80000000u) ? -1.0f : 1.0f;
    if (fabsf(a) <= fabsf(b)) {
        da = sb;
        db = 0.0f;
    } else {
        da = 0.0f;
        db = sa;
    }
}

template <int NLOG, int RLOG>
__global__ __launch_bounds__((Geom<NLOG, RLOG>::WG)) void wbp_bwd_kernel(
    CodeDev code, const float* __restrict__ llr, int64_t B, int T, float lmax, const float* __restrict__ W,
    float* __restrict__ saved, const float* __restrict__ dlam, int dlam_iters, float* __restrict__ dllr) {
    using G = Geom<NLOG, RLOG>;
    constexpr int n = G::n, N = G::N, V = G::V, KL = G::NWIN - 1;
    __shared__ float tb[G::TAB.words];

    const int tid = lid_x();
    const int t = (G::T < 64) ? (tid & (G::T - 1)) : tid;
    const int slot = (G::T < 64) ? (tid >> G::P) : 0;
    const int64_t frame = gid_x() * G::FPW + slot;
    if (G::T < 64 && frame >= B) return;

    int bfrom[G::NB > 0 ? G::NB : 1], bto[G::NB > 0 ? G::NB : 1];
    static_for<0, G::NB>([&](auto J) {
        constexpr int j = decltype(J)::value;
        bfrom[j] = lds_base<G, j, j>(t, slot);
        bto[j] = lds_base<G, j, j + 1>(t, slot);
    });

    float aL[n + 1][V];
    float aR[n + 1][V];
#pragma unroll
    for (int s = 0; s <= n; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            aL[s][v] = 0.0f;
            aR[s][v] = 0.0f;
        }
    float prior[V], chanc[V], chraw[V];
    {
        const int ib = idx_base<G, 0>(t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int i = ib + v;
            prior[v] = ((code.frozen_bits[i >> 5] >> (i & 31)) & 1u) ? lmax : 0.0f;
        }
    }
    {
        const int ib = idx_base<G, KL>(t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            chraw[v] = llr[frame * N + ib + (v << G::wbase(KL))];
            chanc[v] = clipf(chraw[v], lmax);
        }
    }
    float* S = saved + (size_t)frame * T * 2 * n * N;

    for (int it = T - 1; it >= 0; --it) {
        // the loss reads LLR(u) after this iteration (every iteration, or only
        // the last); row 0 of L feeds nothing else, so its adjoint is d loss / d lambda
        if (dlam_iters == T || it == T - 1) {
            const int ib = idx_base<G, 0>(t);
            const float* dl = dlam + ((size_t)frame * dlam_iters + (dlam_iters == T ? it : 0)) * N;
#pragma unroll
            for (int v = 0; v < V; ++v) aL[0][v] = dl[ib + v];
        }
        const float* Wit = W + (size_t)it * 2 * n * N;
        float* St = S + (size_t)it * 2 * n * N;
        const float* Sprev = S + (size_t)(it > 0 ? it - 1 : 0) * 2 * n * N;
        // ---------------- undo the L sweep: columns 0..n-1
        static_for<0, G::NWIN>([&](auto KC) {
            constexpr int k = decltype(KC)::value;
            if constexpr (k > 0) {
                transpose_row<G, k - 1, k - 1, k, false>(aL[G::cbeg(k)], tb, bfrom[k - 1], bto[k - 1]);
            }
            const int ib = idx_base<G, k>(t);
            static_for<G::cbeg(k), G::cend(k)>([&](auto SC) {
                constexpr int s = decltype(SC)::value;
                constexpr int q = s - G::wbase(k);
                constexpr int wb = G::wbase(k);
                float A[V], Rr[V], Wr[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int off = ib + (v << wb);
                    A[v] = (s + 1 == n) ? chanc[v] : St[(size_t)(1 * n + s + 1) * N + off];
                    Rr[v] = (s == 0) ? prior[v] : St[(size_t)(0 * n + s - 1) * N + off];
                    Wr[v] = Wit[(size_t)(1 * n + s) * N + off];
                }
                float dWv[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v & (1 << q)) continue;
                    const int v2 = v | (1 << q);
                    const float a1 = A[v], a2 = A[v2], r1 = Rr[v], r2 = Rr[v2];
                    const float wi = Wr[v], wj = Wr[v2];
                    const float bi = a2 + r2;
                    const float gi = g_ms(a1, bi), gj = g_ms(r1, a1);
                    const float pi = wi * gi, pj = __fmaf_rn(wj, gj, a2);
                    const float di = (fabsf(pi) <= lmax) ? aL[s][v] : 0.0f;
                    const float dj = (fabsf(pj) <= lmax) ? aL[s][v2] : 0.0f;
                    aL[s][v] = 0.0f;
                    aL[s][v2] = 0.0f;
                    dWv[v] = di * gi;
                    dWv[v2] = dj * gj;
                    float ga, gb;
                    g_partials(a1, bi, ga, gb);
                    const float ci = di * wi;
                    aL[s + 1][v] = aL[s + 1][v] + ci * ga;
                    aL[s + 1][v2] = aL[s + 1][v2] + ci * gb;
                    if (s > 0) aR[s][v2] = aR[s][v2] + ci * gb;
                    g_partials(r1, a1, ga, gb);
                    const float cj = dj * wj;
                    if (s > 0) aR[s][v] = aR[s][v] + cj * ga;
                    aL[s + 1][v] = aL[s + 1][v] + cj * gb;
                    aL[s + 1][v2] = aL[s + 1][v2] + dj;
                }
                // L^t_s is no longer read: its slot takes the weight gradient
#pragma unroll
                for (int v = 0; v < V; ++v) St[(size_t)(1 * n + s) * N + ib + (v << wb)] = dWv[v];
            });
        });
        // ---------------- undo the R sweep: columns n-1..0
        static_for_rev<0, G::NWIN>([&](auto KC) {
            constexpr int k = decltype(KC)::value;
            if constexpr (k < G::NWIN - 1) {
                transpose_row<G, k, k + 1, k, true>(aR[G::cend(k)], tb, bto[k], bfrom[k]);
            }
            const int ib = idx_base<G, k>(t);
            static_for_rev<G::cbeg(k), G::cend(k)>([&](auto SC) {
                constexpr int s = decltype(SC)::value;
                constexpr int q = s - G::wbase(k);
                constexpr int wb = G::wbase(k);
                float Lp[V], Rr[V], Wr[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int off = ib + (v << wb);
                    Rr[v] = (s == 0) ? prior[v] : St[(size_t)(0 * n + s - 1) * N + off];
                    Lp[v] = (s + 1 == n) ? chanc[v] : (it == 0 ? 0.0f : Sprev[(size_t)(1 * n + s + 1) * N + off]);
                    Wr[v] = Wit[(size_t)(0 * n + s) * N + off];
                }
                float dWv[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v & (1 << q)) continue;
                    const int v2 = v | (1 << q);
                    const float r1 = Rr[v], r2 = Rr[v2], l1 = Lp[v], l2 = Lp[v2];
                    const float wi = Wr[v], wj = Wr[v2];
                    const float bi = l2 + r2;
                    const float gi = g_ms(r1, bi), gj = g_ms(r1, l1);
                    const float pi = wi * gi, pj = __fmaf_rn(wj, gj, r2);
                    const float di = (fabsf(pi) <= lmax) ? aR[s + 1][v] : 0.0f;
                    const float dj = (fabsf(pj) <= lmax) ? aR[s + 1][v2] : 0.0f;
                    aR[s + 1][v] = 0.0f;
                    aR[s + 1][v2] = 0.0f;
                    dWv[v] = di * gi;
                    dWv[v2] = dj * gj;
                    float ga, gb;
                    g_partials(r1, bi, ga, gb);
                    const float ci = di * wi;
                    if (s > 0) aR[s][v] = aR[s][v] + ci * ga;
                    aL[s + 1][v2] = aL[s + 1][v2] + ci * gb;
                    if (s > 0) aR[s][v2] = aR[s][v2] + ci * gb;
                    g_partials(r1, l1, ga, gb);
                    const float cj = dj * wj;
                    if (s > 0) aR[s][v] = aR[s][v] + cj * ga;
                    aL[s + 1][v] = aL[s + 1][v] + cj * gb;
                    if (s > 0) aR[s][v2] = aR[s][v2] + dj;
                }
                // R^t_{s+1} is no longer read: its slot takes the weight gradient
#pragma unroll
                for (int v = 0; v < V; ++v) St[(size_t)(0 * n + s) * N + ib + (v << wb)] = dWv[v];
            });
        });
    }
    if (dllr) {
        const int ib = idx_base<G, KL>(t);
#pragma unroll
        for (int v = 0; v < V; ++v)
            dllr[frame * N + ib + (v << G::wbase(KL))] = (fabsf(chraw[v]) <= lmax) ? aL[n][v] : 0.0f;
    }
}

using BwdFn = void (*)(CodeDev, const float*, int64_t, int, float, const float*, float*, const float*, int, float*);

struct BwdEntry {
    BwdFn fn;
    int wg, fpw;
};

template <int NL, int RL>
constexpr BwdEntry make_bwd() {
    return BwdEntry{&wbp_bwd_kernel<NL, RL>, Geom<NL, RL>::WG, Geom<NL, RL>::FPW};
}

const BwdEntry* lookup_bwd(int n, int r) {
    static const BwdEntry table[13][4] = {
        {}, {}, {},
        {{}, {}, make_bwd<3, 2>(), make_bwd<3, 3>()},
        {{}, {}, make_bwd<4, 2>(), make_bwd<4, 3>()},
        {{}, {}, make_bwd<5, 2>(), make_bwd<5, 3>()},
        {{}, {}, make_bwd<6, 2>(), make_bwd<6, 3>()},
        {{}, {}, make_bwd<7, 2>(), make_bwd<7, 3>()},
        {{}, {}, make_bwd<8, 2>(), make_bwd<8, 3>()},
        {{}, {}, make_bwd<9, 2>(), make_bwd<9, 3>()},
        {{}, {}, make_bwd<10, 2>(), make_bwd<10, 3>()},
        {{}, {}, make_bwd<11, 2>(), make_bwd<11, 3>()},
        {{}, {}, make_bwd<12, 2>(), make_bwd<12, 3>()},
    };
    if (n < 3 || n > 12 || r < 2 || r > 3) return nullptr;
    return &table[n][r];
}

}  // namespace bp

namespace {

// dW[q] = sum over frames, in frame order, of the per-frame gradients
__global__ __launch_bounds__(256) void wbp_reduce_kernel(const float* __restrict__ part, int64_t B, int64_t P,
                                                         float* __restrict__ dW) {
    const int64_t q = gid_x() * wg_size_x() + lid_x();
    if (q >= P) return;
    double acc = 0.0;
    for (int64_t f = 0; f < B; ++f) acc += (double)part[f * P + q];
    dW[q] = (float)acc;
}

// per-frame loss sum_i softplus((2u_i - 1) lambda_i) * scale over non-frozen i, and
// d loss / d lambda_i = scale (2u_i - 1) sigmoid((2u_i - 1) lambda_i); in double
__global__ __launch_bounds__(256) void wbp_bce_kernel(CodeDev code, const float* __restrict__ lam,
                                                      const uint8_t* __restrict__ u, int64_t B, double scale,
                                                      float* __restrict__ loss, float* __restrict__ dlam) {
    __shared__ double red[256 / 64];
    const int64_t f = gid_x();
    const int N = code.N;
    double acc = 0.0;
    for (int i = lid_x(); i < N; i += wg_size_x()) {
        const bool fr = (code.frozen_bits[i >> 5] >> (i & 31)) & 1u;
        float d = 0.0f;
        if (!fr) {
            const double s = u[f * N + i] ? 1.0 : -1.0;
            const double z = s * (double)lam[f * N + i];
            acc += z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
            const double sig = 1.0 / (1.0 + exp(-z));
            d = (float)(scale * s * sig);
        }
        dlam[f * N + i] = d;
    }
    if (loss) {
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if ((lid_x() & 63) == 0) red[lid_x() >> 6] = acc;
        __syncthreads();
        if (lid_x() == 0) {
            double tot = 0.0;
            for (int w = 0; w < (int)(wg_size_x() / 64); ++w) tot += red[w];
            loss[f] = (float)(tot * scale);
        }
    }
}

// per-iteration loss of frame f (one block): LLR(u) after iteration t = saved
// L row 0 of iteration t + the frozen prior (0 on the non-frozen positions the
// loss reads); the loss sums over iterations and positions in double
__global__ __launch_bounds__(256) void wbp_bce_multi_kernel(CodeDev code, const float* __restrict__ saved,
                                                            const uint8_t* __restrict__ u, int T, double scale,
                                                            float* __restrict__ loss, float* __restrict__ dlam) {
    __shared__ double red[256 / 64];
    const int64_t f = gid_x();
    const int N = code.N, n = code.n;
    double acc = 0.0;
    for (int t = 0; t < T; ++t) {
        const float* lrow = saved + (((size_t)f * T + t) * 2 * n + n) * N;
        float* drow = dlam + ((size_t)f * T + t) * N;
        for (int i = lid_x(); i < N; i += wg_size_x()) {
            const bool fr = (code.frozen_bits[i >> 5] >> (i & 31)) & 1u;
            float d = 0.0f;
            if (!fr) {
                const float lam = lrow[i] + 0.0f;
                const double s = u[f * N + i] ? 1.0 : -1.0;
                const double z = s * (double)lam;
                acc += z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
                const double sig = 1.0 / (1.0 + exp(-z));
                d = (float)(scale * s * sig);
            }
            drow[i] = d;
        }
    }
    if (loss) {
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if ((lid_x() & 63) == 0) red[lid_x() >> 6] = acc;
        __syncthreads();
        if (lid_x() == 0) {
            double tot = 0.0;
            for (int w = 0; w < (int)(wg_size_x() / 64); ++w) tot += red[w];
            loss[f] = (float)(tot * scale);
        }
    }
}

constexpr int kFrameLossMaxT = 256;

// Frame-level losses of frame f (one workgroup), from S_t = sum over the
// non-frozen i of softplus((2u_i - 1) lambda_{t,i}), lambda_{t,i} = saved L row
// 0 of iteration t plus the frozen prior (0 where the loss reads).  With the
// bits taken as independent, q_t = 1 - e^{-S_t} is the probability that some
// decision after iteration t is wrong, and P_u = prod_{t<=u} q_t that the frame
// is still undecided after iteration u.
//   ITER = false: loss = P_T, the probability that no iteration gets the
//     frame right (a smooth stand-in for a BP failure within T iterations);
//   ITER = true:  loss = sum_{u<T} P_u + c P_T, the expected number of
//     iterations beyond the first of an early-stopping decoder plus c per
//     frame still undecided after T (c = fail_weight).
// d loss / d lambda_{t,i} = scale * d loss / d S_t * (2u_i - 1)
// sigmoid((2u_i - 1) lambda_{t,i}), where d loss / d S_t = e^{-S_t} times the
// sum of the products that hold q_t, with q_t taken out.  All in double.
template <bool ITER>
__global__ __launch_bounds__(256) void wbp_frame_loss_kernel(CodeDev code, const float* __restrict__ saved,
                                                             const uint8_t* __restrict__ u, int T, double scale,
                                                             double fail_weight, float* __restrict__ loss,
                                                             float* __restrict__ dlam) {
    __shared__ double red[256 / 64];
    __shared__ double S[kFrameLossMaxT];
    __shared__ double q[kFrameLossMaxT];
    const int64_t f = gid_x();
    const int N = code.N, n = code.n;
    const int nw = wg_size_x() / 64;
    for (int t = 0; t < T; ++t) {
        const float* lrow = saved + (((size_t)f * T + t) * 2 * n + n) * N;
        double acc = 0.0;
        for (int i = lid_x(); i < N; i += wg_size_x()) {
            if ((code.frozen_bits[i >> 5] >> (i & 31)) & 1u) continue;
            const float lam = lrow[i] + 0.0f;
            const double z = (u[f * N + i] ? 1.0 : -1.0) * (double)lam;
            acc += z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
        }
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if ((lid_x() & 63) == 0) red[lid_x() >> 6] = acc;
        __syncthreads();
        if (lid_x() == 0) {
            double tot = 0.0;
            for (int w = 0; w < nw; ++w) tot += red[w];
            S[t] = tot;
            q[t] = -expm1(-tot);
        }
        __syncthreads();
    }
    if (loss && lid_x() == 0) {
        double F = 1.0;
        for (int t = 0; t < T; ++t) F *= q[t];
        double L = F;
        if (ITER) {
            L = 0.0;
            for (int v = 0; v < T - 1; ++v) {
                double P = 1.0;
                for (int t = 0; t <= v; ++t) P *= q[t];
                L += P;
            }
            L += fail_weight * F;
        }
        loss[f] = (float)(L * scale);
    }
    for (int t = 0; t < T; ++t) {
        double dS;
        if (!ITER) {
            dS = exp(-S[t]);
            for (int t2 = 0; t2 < T; ++t2)
                if (t2 != t) dS *= q[t2];
        } else {
            double acc = 0.0;
            for (int v = t; v < T - 1; ++v) {
                double P = 1.0;
                for (int t2 = 0; t2 <= v; ++t2)
                    if (t2 != t) P *= q[t2];
                acc += P;
            }
            double PT = 1.0;
            for (int t2 = 0; t2 < T; ++t2)
                if (t2 != t) PT *= q[t2];
            acc += fail_weight * PT;
            dS = exp(-S[t]) * acc;
        }
        const float* lrow = saved + (((size_t)f * T + t) * 2 * n + n) * N;
        float* drow = dlam + ((size_t)f * T + t) * N;
        for (int i = lid_x(); i < N; i += wg_size_x()) {
            float d = 0.0f;
            if (!((code.frozen_bits[i >> 5] >> (i & 31)) & 1u)) {
                const float lam = lrow[i] + 0.0f;
                const double sg = u[f * N + i] ? 1.0 : -1.0;
                const double z = sg * (double)lam;
                const double sig = 1.0 / (1.0 + exp(-z));
                d = (float)(scale * dS * sg * sig);
            }
            drow[i] = d;
        }
    }
}

// W[t][d][s][i] = Wc[t][d][s]: one weight per stage column spread over its nodes
__global__ __launch_bounds__(256) void wbp_expand_columns_kernel(const float* __restrict__ wc, int64_t cols, int N,
                                                                 float* __restrict__ w) {
    const int64_t q = gid_x() * wg_size_x() + lid_x();
    if (q >= cols * N) return;
    w[q] = wc[q / N];
}

// dWc[c] = sum over the N nodes of column c, in node order, in double: the
// gradient of a weight shared by the whole column
__global__ __launch_bounds__(256) void wbp_sum_columns_kernel(const float* __restrict__ dw, int64_t cols, int N,
                                                              float* __restrict__ dwc) {
    const int64_t c = gid_x() * wg_size_x() + lid_x();
    if (c >= cols) return;
    double acc = 0.0;
    for (int i = 0; i < N; ++i) acc += (double)dw[c * N + i];
    dwc[c] = (float)acc;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t count,
                                                   float lr, float b1, float b2, float eps, float c1, float c2,
                                                   float lo, float hi) {
    const int64_t q = gid_x() * wg_size_x() + lid_x();
    if (q >= count) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / c1, vh = vq / c2;
    w[q] = fminf(fmaxf(w[q] - lr * mh / (sqrtf(vh) + eps), lo), hi);
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

extern "C" polar_status wbp_forward(const polar_code* code, const float* llr, int64_t B, const float* W, int32_t T,
                                    float llr_max, int32_t variant, float* llr_u, uint8_t* u_hat, float* saved,
                                    hipStream_t stream) {
    if (!code || (B > 0 && (!llr || !W || !llr_u || !u_hat)))
        return set_error(POLAR_ERR_INVALID_ARG, "wbp_forward: null argument");
    if (B < 0 || T < 1 || !(llr_max > 0.0f)) return set_error(POLAR_ERR_INVALID_ARG, "wbp_forward: bad sizes");
    if (variant != 0 && !bp_variant_supported(code->n, variant))
        return set_error(POLAR_ERR_INVALID_ARG, "wbp_forward: unknown variant");
    polar_status st = launch_bp_save(code, llr, B, T, llr_max, W, variant, u_hat, llr_u, nullptr, saved, stream);
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status wbp_bce(const polar_code* code, const float* llr_u, const uint8_t* u_true, int64_t B,
                                double scale, float* loss, float* dlam, hipStream_t stream) {
    if (!code || (B > 0 && (!llr_u || !u_true || !dlam))) return set_error(POLAR_ERR_INVALID_ARG, "wbp_bce: null argument");
    if (B < 0) return set_error(POLAR_ERR_INVALID_ARG, "wbp_bce: bad batch");
    if (B == 0) return ok_status();
    hipLaunchKernelGGL(wbp_bce_kernel, dim3((unsigned)B), dim3(256), 0, stream, code->dev(), llr_u, u_true, B, scale,
                       loss, dlam);
    polar_status st = hip_check(hipGetLastError(), "wbp_bce launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status wbp_bce_multi(const polar_code* code, const float* saved, const uint8_t* u_true, int64_t B,
                                      int32_t T, double scale, float* loss, float* dlam, hipStream_t stream) {
    if (!code || (B > 0 && (!saved || !u_true || !dlam)))
        return set_error(POLAR_ERR_INVALID_ARG, "wbp_bce_multi: null argument");
    if (B < 0 || T < 1 || B > (int64_t)INT32_MAX) return set_error(POLAR_ERR_INVALID_ARG, "wbp_bce_multi: bad sizes");
    if (B == 0) return ok_status();
    hipLaunchKernelGGL(wbp_bce_multi_kernel, dim3((unsigned)B), dim3(256), 0, stream, code->dev(), saved, u_true, T,
                       scale, loss, dlam);
    polar_status st = hip_check(hipGetLastError(), "wbp_bce_multi launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status wbp_backward(const polar_code* code, const float* llr, int64_t B, const float* W, int32_t T,
                                     float llr_max, int32_t variant, float* saved, const float* dlam,
                                     int32_t dlam_iters, float* dW, float* dllr, hipStream_t stream) {
    if (!code || !W || !dW || (B > 0 && (!llr || !saved || !dlam)))
        return set_error(POLAR_ERR_INVALID_ARG, "wbp_backward: null argument");
    if (B < 0 || T < 1 || !(llr_max > 0.0f)) return set_error(POLAR_ERR_INVALID_ARG, "wbp_backward: bad sizes");
    if (dlam_iters != 1 && dlam_iters != T)
        return set_error(POLAR_ERR_INVALID_ARG, "wbp_backward: dlam_iters must be 1 or T");
    const int v = variant ? variant : bp_default_variant(code->n);
    const bp::BwdEntry* e = bp::lookup_bwd(code->n, v);
    if (!e) return set_error(POLAR_ERR_UNSUPPORTED, "wbp_backward: no kernel variant for this block length");
    const int64_t P = (int64_t)T * 2 * code->n * code->N;
    if (B > 0) {
        const int64_t blocks = (B + e->fpw - 1) / e->fpw;
        hipLaunchKernelGGL(e->fn, dim3((unsigned)blocks), dim3(e->wg), 0, stream, code->dev(), llr, B, T, llr_max, W,
                           saved, dlam, dlam_iters, dllr);
        polar_status st = hip_check(hipGetLastError(), "wbp_bwd launch");
        if (st != POLAR_OK) return st;
    }
    hipLaunchKernelGGL(wbp_reduce_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, saved, B, P, dW);
    polar_status st = hip_check(hipGetLastError(), "wbp_reduce launch");
    return st == POLAR_OK ? ok_status() : st;
}

static polar_status adam_launch(float* w, const float* g, float* m, float* v, int64_t count, int32_t step, float lr,
                                float beta1, float beta2, float eps, float lo, float hi, hipStream_t stream) {
    if (!w || !g || !m || !v || count < 0 || step < 1) return set_error(POLAR_ERR_INVALID_ARG, "polar_adam_step: bad argument");
    if (!(lo <= hi)) return set_error(POLAR_ERR_INVALID_ARG, "polar_adam_step_bounded: need lo <= hi");
    if (count == 0) return ok_status();
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, w, g, m, v, count, lr,
                       beta1, beta2, eps, c1, c2, lo, hi);
    polar_status st = hip_check(hipGetLastError(), "adam launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status polar_adam_step(float* w, const float* g, float* m, float* v, int64_t count, int32_t step,
                                        float lr, float beta1, float beta2, float eps, hipStream_t stream) {
    return adam_launch(w, g, m, v, count, step, lr, beta1, beta2, eps, -INFINITY, INFINITY, stream);
}

extern "C" polar_status polar_adam_step_bounded(float* w, const float* g, float* m, float* v, int64_t count,
                                                int32_t step, float lr, float beta1, float beta2, float eps, float lo,
                                                float hi, hipStream_t stream) {
    return adam_launch(w, g, m, v, count, step, lr, beta1, beta2, eps, lo, hi, stream);
}

static polar_status frame_loss_launch(const char* who, bool iter, const polar_code* code, const float* saved,
                                      const uint8_t* u_true, int64_t B, int32_t T, double fail_weight, double scale,
                                      float* loss, float* dlam, hipStream_t stream) {
    if (!code || (B > 0 && (!saved || !u_true || !dlam)))
        return set_error(POLAR_ERR_INVALID_ARG, std::string(who) + ": null argument");
    if (B < 0 || T < 1 || T > kFrameLossMaxT || B > (int64_t)INT32_MAX)
        return set_error(POLAR_ERR_INVALID_ARG, std::string(who) + ": bad sizes (1 <= T <= 256)");
    if (!(fail_weight >= 0.0)) return set_error(POLAR_ERR_INVALID_ARG, std::string(who) + ": fail_weight < 0");
    if (B == 0) return ok_status();
    if (iter)
        hipLaunchKernelGGL(wbp_frame_loss_kernel<true>, dim3((unsigned)B), dim3(256), 0, stream, code->dev(), saved,
                           u_true, T, scale, fail_weight, loss, dlam);
    else
        hipLaunchKernelGGL(wbp_frame_loss_kernel<false>, dim3((unsigned)B), dim3(256), 0, stream, code->dev(), saved,
                           u_true, T, scale, fail_weight, loss, dlam);
    polar_status st = hip_check(hipGetLastError(), "frame loss launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status wbp_frame_loss(const polar_code* code, const float* saved, const uint8_t* u_true, int64_t B,
                                       int32_t T, double scale, float* loss, float* dlam, hipStream_t stream) {
    return frame_loss_launch("wbp_frame_loss", false, code, saved, u_true, B, T, 0.0, scale, loss, dlam, stream);
}

extern "C" polar_status wbp_iteration_loss(const polar_code* code, const float* saved, const uint8_t* u_true,
                                           int64_t B, int32_t T, double fail_weight, double scale, float* loss,
                                           float* dlam, hipStream_t stream) {
    return frame_loss_launch("wbp_iteration_loss", true, code, saved, u_true, B, T, fail_weight, scale, loss, dlam,
                             stream);
}

extern "C" polar_status wbp_column_weights(const polar_code* code, const float* Wc, int32_t T, float* W,
                                           hipStream_t stream) {
    if (!code || !Wc || !W) return set_error(POLAR_ERR_INVALID_ARG, "wbp_column_weights: null argument");
    if (T < 1) return set_error(POLAR_ERR_INVALID_ARG, "wbp_column_weights: T < 1");
    const int64_t cols = (int64_t)T * 2 * code->n, tot = cols * code->N;
    hipLaunchKernelGGL(wbp_expand_columns_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, Wc, cols,
                       code->N, W);
    polar_status st = hip_check(hipGetLastError(), "wbp_column_weights launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status wbp_column_grad(const polar_code* code, const float* dW, int32_t T, float* dWc,
                                        hipStream_t stream) {
    if (!code || !dW || !dWc) return set_error(POLAR_ERR_INVALID_ARG, "wbp_column_grad: null argument");
    if (T < 1) return set_error(POLAR_ERR_INVALID_ARG, "wbp_column_grad: T < 1");
    const int64_t cols = (int64_t)T * 2 * code->n;
    hipLaunchKernelGGL(wbp_sum_columns_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, stream, dW, cols,
                       code->N, dWc);
    polar_status st = hip_check(hipGetLastError(), "wbp_column_grad launch");
    return st == POLAR_OK ? ok_status() : st;
}
