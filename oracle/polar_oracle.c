/*
 * polar_oracle.c -- plain CPU reference of the hybrid BP -> CA-SCL polar
 * decoder of Cammerer et al., "Combining Belief Propagation and Successive
 * Cancellation List Decoding of Polar Codes on a GPU Platform".
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only
 * the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  The product path never links, imports or calls it,
 * and it shares no code, header, table or constant generator with the GPU
 * library.
 *
 * The file is compiled twice:
 *   REAL=double  reference arithmetic (message values, gradients, statistics);
 *   REAL=float   the paper's own 32-bit precision (Sec. I: the authors' decoder
 *                computes in 32-bit floating point).  Where a floating-point
 *                value decides an integer (a hard decision, the early-stop
 *                test, the iteration count, which list path survives) the GPU
 *                result is compared with the REAL=float oracle, bit for bit.
 *
 * Everything is written for clarity, not speed: plain loops, one frame at a
 * time, no blocking, fusion or reordering beyond what each definition states.
 * Compile with -ffp-contract=off so that every "+" and "*" is one IEEE
 * operation; fused multiply-adds appear only where written as FMA().
 *
 * Conventions (Sec. II): N = 2^n, x = u * F^{(x)n} with F = [[1,0],[1,1]],
 * indices in natural order; frozen[i] = 1 marks a frozen position (value 0);
 * the k = K + c non-frozen positions carry K info bits followed by c CRC bits
 * in ascending index order; LLR = ln P(y|0)/P(y|1), so LLR > 0 favours bit 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_F32
typedef float real;
#define FMA(a, b, c) fmaf((a), (b), (c))
#else
typedef double real;
#define FMA(a, b, c) fma((a), (b), (c))
#endif

/* ------------------------------------------------------------------------ */
/* Small helpers                                                             */
/* ------------------------------------------------------------------------ */

static int ilog2(int N) {
    int n = 0;
    while ((1 << n) < N) n++;
    return n;
}

static int ctz_int(int v) {
    int c = 0;
    while (((v >> c) & 1) == 0) c++;
    return c;
}

/* Hard decision: bit 1 iff the LLR is negative (an LLR of +0 or -0 gives 0). */
static uint8_t hard(real v) { return v < 0 ? 1 : 0; }

static real clip(real v, real m) {
    if (v > m) return m;
    if (v < -m) return -m;
    return v;
}

/* Sign taken from the IEEE sign bit, so -0 counts as negative. */
static real sgn(real v) { return signbit(v) ? (real)-1 : (real)1; }

/* Min-sum rule (Sec. II-B): g(a,b) = sign(a) sign(b) min(|a|,|b|). */
static real g_minsum(real a, real b) {
    real ma = fabs(a), mb = fabs(b);
    real m = (ma <= mb) ? ma : mb;
    return (signbit(a) != signbit(b)) ? -m : m;
}

/* Exact rule (Sec. II-B): g(a,b) = ln((1 + e^{a+b}) / (e^a + e^b)).  In BP
 * its arguments are bounded by the clipping (|a| <= 20, |b| <= 40), so the
 * definition is evaluated as written, in double. */
static real g_exact_bounded(real a, real b) {
    double A = a, B = b;
    return (real)log((1.0 + exp(A + B)) / (exp(A) + exp(B)));
}

/* The same function for unbounded arguments (SC / SCL work on unclipped
 * LLRs).  Identity used: ln((1+e^{a+b})/(e^a+e^b)) =
 *   sign(a)sign(b)min(|a|,|b|) + ln(1+e^{-|a+b|}) - ln(1+e^{-|a-b|}). */
static real g_exact_stable(real a, real b) {
    double A = a, B = b;
    double m = fabs(A) < fabs(B) ? fabs(A) : fabs(B);
    double s = ((A < 0) != (B < 0)) ? -1.0 : 1.0;
    return (real)(s * m + log1p(exp(-fabs(A + B))) - log1p(exp(-fabs(A - B))));
}

/* softplus(z) = ln(1 + e^z), evaluated without overflow. */
static double softplus(double z) {
    return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
}

/* ------------------------------------------------------------------------ */
/* Code construction by Gaussian approximation (density evolution).          */
/* The paper takes the frozen vector as given (Sec. II); the workloads build */
/* it with the Gaussian approximation of Chung, Richardson and Urbanke       */
/* (2001), as applied to polar codes by Trifonov (2012).                     */
/* ------------------------------------------------------------------------ */

/* ln phi(x) with the two-piece approximation of Chung et al. */
static double ga_ln_phi(double x) {
    if (x <= 0.0) return 0.0;
    if (x < 10.0) return -0.4527 * pow(x, 0.86) + 0.0218;
    return 0.5 * log(M_PI / x) - 0.25 * x + log(1.0 - 10.0 / (7.0 * x));
}

/* phi^{-1}, given ln y: the smallest x with ln phi(x) <= ln y.  The first
 * piece is inverted in closed form; on x >= 10 the second piece is monotone
 * decreasing and is inverted by bisection. */
static double ga_phi_inv_ln(double lny) {
    double at10 = -0.4527 * pow(10.0, 0.86) + 0.0218;
    if (lny >= 0.0) return 0.0;
    if (lny >= at10) return pow((0.0218 - lny) / 0.4527, 1.0 / 0.86);
    double lo = 10.0, hi = 20.0;
    while (ga_ln_phi(hi) > lny) hi *= 2.0;
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (ga_ln_phi(mid) > lny) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double orc_sigma2(double ebn0_db, double rate) {
    return 1.0 / (2.0 * rate * pow(10.0, ebn0_db / 10.0));
}

/* Mean LLR of each of the N bit channels.  Start from the channel mean
 * 2/sigma^2; each of the n polarisation steps maps a mean m to the pair
 *   (check side)    phi^{-1}(1 - (1 - phi(m))^2)
 *   (variable side) 2 m,
 * appended as the next least significant index bit, so the first step decides
 * the most significant bit of the index (u's first half is decoded through the
 * check-node side). */
void orc_ga_means(int N, double sigma2, double* m_out) {
    int n = ilog2(N);
    double* cur = (double*)malloc(sizeof(double) * N);
    double* nxt = (double*)malloc(sizeof(double) * N);
    cur[0] = 2.0 / sigma2;
    int len = 1;
    for (int t = 0; t < n; t++) {
        for (int q = 0; q < len; q++) {
            double m = cur[q];
            double lnp = ga_ln_phi(m);
            double p = exp(lnp);
            /* 1 - (1 - p)^2 = p (2 - p) */
            double ln_check = lnp + log(2.0 - p);
            nxt[2 * q] = ga_phi_inv_ln(ln_check);
            nxt[2 * q + 1] = 2.0 * m;
        }
        len *= 2;
        double* tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(m_out, cur, sizeof(double) * N);
    free(cur);
    free(nxt);
}

/* Frozen mask: the k positions with the largest mean are non-frozen; equal
 * means are ordered by index, the higher index counting as more reliable. */
void orc_ga_frozen(int N, int k, double design_ebn0_db, double rate,
                   uint8_t* frozen_out, double* m_out_or_null) {
    double* m = (double*)malloc(sizeof(double) * N);
    orc_ga_means(N, orc_sigma2(design_ebn0_db, rate), m);
    for (int i = 0; i < N; i++) frozen_out[i] = 1;
    /* k rounds of "pick the best remaining" -- quadratic, but obviously right */
    uint8_t* taken = (uint8_t*)calloc(N, 1);
    for (int r = 0; r < k; r++) {
        int best = -1;
        for (int i = 0; i < N; i++) {
            if (taken[i]) continue;
            if (best < 0 || m[i] > m[best] || (m[i] == m[best] && i > best)) best = i;
        }
        taken[best] = 1;
        frozen_out[best] = 0;
    }
    if (m_out_or_null) memcpy(m_out_or_null, m, sizeof(double) * N);
    free(taken);
    free(m);
}

/* ------------------------------------------------------------------------ */
/* CRC (Sec. II-A: CRC-aided selection, c parity bits).  Polynomial long     */
/* division, most significant bit first, zero initial register, no           */
/* reflection and no final XOR: the c remainder bits of M(x) x^c mod P(x).   */
/* ------------------------------------------------------------------------ */

void orc_crc(const uint8_t* bits, int nbits, int c, uint32_t poly, uint8_t* out) {
    uint64_t reg = 0;
    uint64_t top = 1ull << (c - 1);
    uint64_t mask = (1ull << c) - 1ull;
    for (int i = 0; i < nbits; i++) {
        uint64_t fb = ((reg & top) ? 1u : 0u) ^ (uint64_t)(bits[i] & 1u);
        reg = (reg << 1) & mask;
        if (fb) reg ^= (uint64_t)poly;
    }
    for (int j = 0; j < c; j++) out[j] = (uint8_t)((reg >> (c - 1 - j)) & 1u);
}

/* 1 if the last c of the k non-frozen bits of u equal the CRC of the first
 * K = k - c; always 1 when c == 0. */
static int crc_holds(const uint8_t* u, const uint8_t* frozen, int N, int c, uint32_t poly) {
    if (c == 0) return 1;
    uint8_t* b = (uint8_t*)malloc(N);
    int k = 0;
    for (int i = 0; i < N; i++) if (!frozen[i]) b[k++] = u[i];
    uint8_t* r = (uint8_t*)malloc(c);
    orc_crc(b, k - c, c, poly, r);
    int ok = 1;
    for (int j = 0; j < c; j++) if (r[j] != b[k - c + j]) ok = 0;
    free(r);
    free(b);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Encoder (Sec. II, Fig. 1): x = u G with G = F^{(x)n}.  Stage by stage,    */
/* the butterfly at distance d adds the lower node into the upper one.        */
/* ------------------------------------------------------------------------ */

void orc_polar_transform(const uint8_t* u, int N, uint8_t* x) {
    for (int i = 0; i < N; i++) x[i] = u[i] & 1u;
    for (int d = 1; d < N; d <<= 1)
        for (int i = 0; i < N; i++)
            if ((i & d) == 0) x[i] ^= x[i + d];
}

/* u: K info bits, then their c CRC bits, on the non-frozen positions in
 * ascending order; zeros elsewhere. */
void orc_build_u(const uint8_t* info, int K, int c, uint32_t poly,
                 const uint8_t* frozen, int N, uint8_t* u) {
    uint8_t* b = (uint8_t*)malloc(K + c + 1);
    for (int q = 0; q < K; q++) b[q] = info[q] & 1u;
    if (c > 0) orc_crc(info, K, c, poly, b + K);
    int q = 0;
    for (int i = 0; i < N; i++) u[i] = frozen[i] ? 0 : b[q++];
    free(b);
}

void orc_encode_batch(const uint8_t* info, int64_t B, int K, int c, uint32_t poly,
                      const uint8_t* frozen, int N, uint8_t* u_out, uint8_t* x_out) {
    uint8_t* u = (uint8_t*)malloc(N);
    for (int64_t f = 0; f < B; f++) {
        orc_build_u(info + f * K, K, c, poly, frozen, N, u);
        if (u_out) memcpy(u_out + f * N, u, N);
        orc_polar_transform(u, N, x_out + f * N);
    }
    free(u);
}

/* BPSK over AWGN: s = 1 - 2x, y = s + sigma z, LLR = ln p(y|0)/p(y|1) = 2y/sigma^2
 * (Sec. II-A defines the LLR).  The noise z is an input. */
void orc_channel_llr(const uint8_t* x, const double* z, int64_t count, double sigma2, float* llr) {
    double sigma = sqrt(sigma2);
    for (int64_t i = 0; i < count; i++) {
        double y = (x[i] ? -1.0 : 1.0) + sigma * z[i];
        llr[i] = (float)(2.0 * y / sigma2);
    }
}

/* ------------------------------------------------------------------------ */
/* BP decoder (Sec. II-B, Fig. 2).                                           */
/* Node stages 1..n+1 of the paper are rows 0..n here: row 0 is the u side,  */
/* row n the channel side.  PE column s (0-based) joins rows s and s+1 and    */
/* pairs node i with j = i + 2^s (Fig. 1: the XOR sits on the upper node i).  */
/* Ports (Fig. 2): in1/out1 belong to node i, in2/out2 to node j; R inputs    */
/* come from row s, L inputs from row s+1.                                    */
/*   R sweep, s = 0..n-1:  R[s+1][i] = g(R[s][i], L[s+1][j] + R[s][j])        */
/*                         R[s+1][j] = g(R[s][i], L[s+1][i]) + R[s][j]        */
/*   L sweep, s = n-1..0:  L[s][i]   = g(L[s+1][i], L[s+1][j] + R[s][j])      */
/*                         L[s][j]   = g(R[s][i], L[s+1][i]) + L[s+1][j]      */
/* Init: L[n] = channel LLRs, R[0][i] = LLR_max * f_i, all else 0.           */
/* Output: LLR(u_i) = L[0][i] + R[0][i], LLR(x_i) = L[n][i] + R[n][i].       */
/* Clipping to +-LLR_max is applied to the channel LLRs and to every         */
/* computed PE output.                                                        */
/* Weighted (learned) form: the g term of each output is multiplied by       */
/* W[t][dir][s][node] (dir 0 = R, 1 = L; node = the output node) before the  */
/* "+" and the clipping; the "+" outputs use one fused multiply-add.         */
/* Early stop after each iteration (Sec. II-B): stop = 1 when u_hat G equals */
/* x_hat (re-encoding check), stop = 2 when the CRC of u_hat holds, 0 never. */
/* ok: stop = 2 -> CRC holds; otherwise re-encoding check and CRC both hold. */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, N;
    real* L;   /* (n+1) x N */
    real* R;   /* (n+1) x N */
} bp_state;

static real G(real a, real b, int rule) {
    return rule == 0 ? g_minsum(a, b) : g_exact_bounded(a, b);
}

static void bp_iteration(bp_state* st, int rule, real lmax, const double* Wt /* [2][n][N] or NULL */) {
    int n = st->n, N = st->N;
    real* L = st->L;
    real* R = st->R;
    for (int s = 0; s < n; s++) {
        int d = 1 << s;
        for (int i = 0; i < N; i++) {
            if (i & d) continue;
            int j = i + d;
            real r1 = R[s * N + i], r2 = R[s * N + j];
            real l1 = L[(s + 1) * N + i], l2 = L[(s + 1) * N + j];
            real gi = G(r1, l2 + r2, rule);
            real gj = G(r1, l1, rule);
            if (Wt) {
                real wi = (real)Wt[(0 * n + s) * N + i], wj = (real)Wt[(0 * n + s) * N + j];
                R[(s + 1) * N + i] = clip(wi * gi, lmax);
                R[(s + 1) * N + j] = clip(FMA(wj, gj, r2), lmax);
            } else {
                R[(s + 1) * N + i] = clip(gi, lmax);
                R[(s + 1) * N + j] = clip(gj + r2, lmax);
            }
        }
    }
    for (int s = n - 1; s >= 0; s--) {
        int d = 1 << s;
        for (int i = 0; i < N; i++) {
            if (i & d) continue;
            int j = i + d;
            real r1 = R[s * N + i], r2 = R[s * N + j];
            real l1 = L[(s + 1) * N + i], l2 = L[(s + 1) * N + j];
            real gi = G(l1, l2 + r2, rule);
            real gj = G(r1, l1, rule);
            if (Wt) {
                real wi = (real)Wt[(1 * n + s) * N + i], wj = (real)Wt[(1 * n + s) * N + j];
                L[s * N + i] = clip(wi * gi, lmax);
                L[s * N + j] = clip(FMA(wj, gj, l2), lmax);
            } else {
                L[s * N + i] = clip(gi, lmax);
                L[s * N + j] = clip(gj + l2, lmax);
            }
        }
    }
}

static void bp_init(bp_state* st, const float* llr, const uint8_t* frozen, real lmax) {
    int n = st->n, N = st->N;
    memset(st->L, 0, sizeof(real) * (n + 1) * N);
    memset(st->R, 0, sizeof(real) * (n + 1) * N);
    for (int i = 0; i < N; i++) {
        st->L[n * N + i] = clip((real)llr[i], lmax);
        st->R[i] = frozen[i] ? lmax : (real)0;
    }
}

/* Returns the number of iterations run. */
int orc_bp_frame(const float* llr, int N, const uint8_t* frozen, int c, uint32_t poly,
                 int max_iter, int stop, double llr_max, int rule,
                 const double* W /* [max_iter][2][n][N] or NULL */,
                 uint8_t* u_hat, double* llr_u /* or NULL */, double* llr_x /* or NULL */,
                 uint8_t* ok_out, double* save /* [max_iter][2][n][N] or NULL */) {
    int n = ilog2(N);
    bp_state st;
    st.n = n;
    st.N = N;
    st.L = (real*)malloc(sizeof(real) * (n + 1) * N);
    st.R = (real*)malloc(sizeof(real) * (n + 1) * N);
    uint8_t* uh = (uint8_t*)malloc(N);
    uint8_t* xh = (uint8_t*)malloc(N);
    uint8_t* re = (uint8_t*)malloc(N);
    real lmax = (real)llr_max;
    bp_init(&st, llr, frozen, lmax);
    int it = 0, gcheck = 0, crcok = 0;
    for (int t = 0; t < max_iter; t++) {
        bp_iteration(&st, rule, lmax, W ? W + (size_t)t * 2 * n * N : NULL);
        it = t + 1;
        if (save) {
            double* sv = save + (size_t)t * 2 * n * N;
            for (int s = 0; s < n; s++)
                for (int i = 0; i < N; i++) {
                    sv[(0 * n + s) * N + i] = (double)st.R[(s + 1) * N + i];
                    sv[(1 * n + s) * N + i] = (double)st.L[s * N + i];
                }
        }
        for (int i = 0; i < N; i++) {
            real lu = st.L[i] + st.R[i];
            uh[i] = frozen[i] ? 0 : hard(lu);
            xh[i] = hard(st.L[n * N + i] + st.R[n * N + i]);
        }
        orc_polar_transform(uh, N, re);
        gcheck = memcmp(re, xh, N) == 0;
        crcok = crc_holds(uh, frozen, N, c, poly);
        if ((stop == 1 && gcheck) || (stop == 2 && crcok)) break;
    }
    memcpy(u_hat, uh, N);
    if (llr_u) for (int i = 0; i < N; i++) llr_u[i] = (double)(st.L[i] + st.R[i]);
    if (llr_x) for (int i = 0; i < N; i++) llr_x[i] = (double)(st.L[n * N + i] + st.R[n * N + i]);
    *ok_out = (uint8_t)(stop == 2 ? crcok : (gcheck && crcok));
    free(st.L);
    free(st.R);
    free(uh);
    free(xh);
    free(re);
    return it;
}

void orc_bp_batch(const float* llr, int64_t B, int N, const uint8_t* frozen, int c, uint32_t poly,
                  int max_iter, int stop, double llr_max, int rule, const double* W,
                  uint8_t* u_hat, double* llr_u, int32_t* iters, uint8_t* ok) {
    for (int64_t f = 0; f < B; f++) {
        int it = orc_bp_frame(llr + f * N, N, frozen, c, poly, max_iter, stop, llr_max, rule, W,
                              u_hat + f * N, llr_u ? llr_u + f * N : NULL, NULL, ok + f, NULL);
        if (iters) iters[f] = it;
    }
}

/* ------------------------------------------------------------------------ */
/* SC decoder (Sec. II-A builds SCL on Arikan's bitwise-serial SC).          */
/* Recursive, natural order: with u = (u_a, u_b), x = ((u_a+u_b)G', u_b G'),  */
/* so u_a is decoded from f(top, bottom), then u_b from                      */
/* bottom + (1 - 2 v) top with v = u_a G' the re-encoded first half.          */
/* ------------------------------------------------------------------------ */

static real F(real a, real b, int rule) {
    return rule == 0 ? g_minsum(a, b) : g_exact_stable(a, b);
}

static void sc_rec(const real* lam, int M, const uint8_t* frozen, int off, int rule,
                   uint8_t* u, uint8_t* x_out) {
    if (M == 1) {
        u[off] = frozen[off] ? 0 : hard(lam[0]);
        x_out[0] = u[off];
        return;
    }
    int h = M / 2;
    real* top = (real*)malloc(sizeof(real) * h);
    real* bot = (real*)malloc(sizeof(real) * h);
    uint8_t* v = (uint8_t*)malloc(h);
    uint8_t* w = (uint8_t*)malloc(h);
    for (int e = 0; e < h; e++) top[e] = F(lam[e], lam[e + h], rule);
    sc_rec(top, h, frozen, off, rule, u, v);
    for (int e = 0; e < h; e++) bot[e] = v[e] ? lam[e + h] - lam[e] : lam[e + h] + lam[e];
    sc_rec(bot, h, frozen, off + h, rule, u, w);
    for (int e = 0; e < h; e++) {
        x_out[e] = v[e] ^ w[e];
        x_out[e + h] = w[e];
    }
    free(top);
    free(bot);
    free(v);
    free(w);
}

void orc_sc_frame(const float* llr, int N, const uint8_t* frozen, int rule, uint8_t* u_hat) {
    real* lam = (real*)malloc(sizeof(real) * N);
    uint8_t* x = (uint8_t*)malloc(N);
    for (int i = 0; i < N; i++) lam[i] = (real)llr[i];
    sc_rec(lam, N, frozen, 0, rule, u_hat, x);
    free(lam);
    free(x);
}

/* ------------------------------------------------------------------------ */
/* CA-SCL decoder (Sec. II-A), LLR-based list decoding with path metrics.    */
/* Each path keeps its own copy of the LLR levels (level d: 2^d values,       */
/* d = 0..n-1, level n = the channel) and of the partial sums; a branching    */
/* path is copied whole.  Bit i recomputes levels ctz(i)..0 (all levels for   */
/* i = 0): level ctz(i) by the "g" step with the stored partial sums, the     */
/* rest by f.  Penalties (smaller metric is better):                          */
/*   rule 0: pen(lam, b) = |lam| if b differs from the hard decision, else 0; */
/*   rule 1: pen(lam, b) = ln(1 + e^{-(1-2b) lam}).                            */
/* Frozen bit: no branching, bit 0, metric += pen(lam, 0).                    */
/* Info bit: every path spawns bits 0 and 1, listed parent by parent (the     */
/* parent's position in the list, then bit 0 before bit 1).  The candidates   */
/* ranked first by (metric, parent's position, bit), min(L, 2*len) of them,   */
/* survive: the "L smallest metrics" of the pruned pseudo sort, made a strict */
/* total order so that exactly that many survive.  The pseudo sort discards   */
/* candidates without moving the others, so the survivors form the new list   */
/* in the order in which the candidates were listed.                          */
/* End: the path of smallest (metric, position) whose CRC holds; if none      */
/* holds, the path of smallest (metric, position), reported with crc_ok = 0.  */
/* ------------------------------------------------------------------------ */

typedef struct {
    real* lam;    /* N - 1 values: level d at offset 2^d - 1 */
    uint8_t* ps;  /* N - 1 partial sums, same layout */
    uint8_t* u;   /* N decided bits */
    real pm;
} scl_path;

typedef struct {
    real metric;
    int parent;
    int bit;
} scl_cand;

static int cand_cmp(const void* pa, const void* pb) {
    const scl_cand* a = (const scl_cand*)pa;
    const scl_cand* b = (const scl_cand*)pb;
    if (a->metric < b->metric) return -1;
    if (a->metric > b->metric) return 1;
    if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
    return a->bit - b->bit;
}

/* the order in which the candidates are listed: parent's position, then bit */
static int cand_list_cmp(const void* pa, const void* pb) {
    const scl_cand* a = (const scl_cand*)pa;
    const scl_cand* b = (const scl_cand*)pb;
    if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
    return a->bit - b->bit;
}

static real penalty(real lam, int b, int rule) {
    if (rule == 0) return (b != hard(lam)) ? (real)fabs(lam) : (real)0;
    return (real)softplus(-(1.0 - 2.0 * b) * (double)lam);
}

static void scl_levels(scl_path* p, const real* ch, int n, int i, int rule) {
    int top = (i == 0) ? n - 1 : ctz_int(i);
    for (int d = top; d >= 0; d--) {
        int h = 1 << d;
        const real* src = (d == n - 1) ? ch : p->lam + (2 * h - 1);
        real* dst = p->lam + (h - 1);
        const uint8_t* v = p->ps + (h - 1);
        for (int e = 0; e < h; e++) {
            real a = src[e], b = src[e + h];
            if (d == top && i != 0)
                dst[e] = v[e] ? b - a : b + a;
            else
                dst[e] = F(a, b, rule);
        }
    }
}

static void scl_partial_sums(scl_path* p, int n, int i, uint8_t bit, uint8_t* tmp) {
    int size = 1, d = 0;
    tmp[0] = bit;
    while (d < n && ((i >> d) & 1)) {
        const uint8_t* v = p->ps + (size - 1);
        for (int e = 0; e < size; e++) tmp[e + size] = tmp[e];
        for (int e = 0; e < size; e++) tmp[e] ^= v[e];
        size *= 2;
        d++;
    }
    if (d < n) memcpy(p->ps + (size - 1), tmp, size);
}

static void path_alloc(scl_path* p, int N) {
    p->lam = (real*)calloc(N, sizeof(real));
    p->ps = (uint8_t*)calloc(N, 1);
    p->u = (uint8_t*)calloc(N, 1);
    p->pm = 0;
}

static void path_free(scl_path* p) {
    free(p->lam);
    free(p->ps);
    free(p->u);
}

static void path_copy(scl_path* dst, const scl_path* src, int N) {
    memcpy(dst->lam, src->lam, sizeof(real) * N);
    memcpy(dst->ps, src->ps, N);
    memcpy(dst->u, src->u, N);
    dst->pm = src->pm;
}

/* Returns the number of paths in the final list.  u_hat gets the selected
 * path; all_u / all_pm (optional, L x N and L) get the whole final list in
 * list order. */
int orc_scl_frame(const float* llr, int N, const uint8_t* frozen, const uint8_t* da, int c,
                  uint32_t poly, int L, int rule, uint8_t* u_hat, uint8_t* crc_ok, double* pm_out,
                  uint8_t* all_u, double* all_pm) {
    int n = ilog2(N);
    real* ch = (real*)malloc(sizeof(real) * N);
    for (int i = 0; i < N; i++) ch[i] = (real)llr[i];
    scl_path* cur = (scl_path*)malloc(sizeof(scl_path) * L);
    scl_path* nxt = (scl_path*)malloc(sizeof(scl_path) * L);
    for (int q = 0; q < L; q++) {
        path_alloc(&cur[q], N);
        path_alloc(&nxt[q], N);
    }
    scl_cand* cand = (scl_cand*)malloc(sizeof(scl_cand) * 2 * L);
    real* lam_i = (real*)malloc(sizeof(real) * L);
    uint8_t* tmp = (uint8_t*)malloc(N);
    int len = 1;
    for (int i = 0; i < N; i++) {
        for (int q = 0; q < len; q++) {
            scl_levels(&cur[q], ch, n, i, rule);
            lam_i[q] = cur[q].lam[0];
        }
        if (frozen[i]) {
            for (int q = 0; q < len; q++) {
                cur[q].u[i] = 0;
                cur[q].pm = cur[q].pm + penalty(lam_i[q], 0, rule);
            }
        } else if (da && da[i]) {
            /* decision-aided position (Sec. II-A): every path takes its own hard
               decision; the list neither branches nor reorders */
            for (int q = 0; q < len; q++) {
                int b = lam_i[q] < 0 ? 1 : 0;
                cur[q].u[i] = (uint8_t)b;
                cur[q].pm = cur[q].pm + penalty(lam_i[q], b, rule);
            }
        } else {
            int nc = 0;
            for (int q = 0; q < len; q++)
                for (int b = 0; b < 2; b++) {
                    cand[nc].metric = cur[q].pm + penalty(lam_i[q], b, rule);
                    cand[nc].parent = q;
                    cand[nc].bit = b;
                    nc++;
                }
            qsort(cand, nc, sizeof(scl_cand), cand_cmp);
            int keep = nc < L ? nc : L;
            /* the survivors, back in the order they were listed */
            qsort(cand, keep, sizeof(scl_cand), cand_list_cmp);
            for (int q = 0; q < keep; q++) {
                path_copy(&nxt[q], &cur[cand[q].parent], N);
                nxt[q].u[i] = (uint8_t)cand[q].bit;
                nxt[q].pm = cand[q].metric;
            }
            scl_path* t = cur; cur = nxt; nxt = t;
            len = keep;
        }
        for (int q = 0; q < len; q++) scl_partial_sums(&cur[q], n, i, cur[q].u[i], tmp);
    }
    int best = -1, best_ok = 0;
    for (int q = 0; q < len; q++) {
        int ok = crc_holds(cur[q].u, frozen, N, c, poly);
        if (ok && (!best_ok || cur[q].pm < cur[best].pm)) {
            best = q;
            best_ok = 1;
        }
    }
    if (!best_ok) {
        best = 0;
        for (int q = 1; q < len; q++) if (cur[q].pm < cur[best].pm) best = q;
    }
    memcpy(u_hat, cur[best].u, N);
    *crc_ok = (uint8_t)best_ok;
    if (pm_out) *pm_out = (double)cur[best].pm;
    for (int q = 0; q < len; q++) {
        if (all_u) memcpy(all_u + (size_t)q * N, cur[q].u, N);
        if (all_pm) all_pm[q] = (double)cur[q].pm;
    }
    for (int q = 0; q < L; q++) {
        path_free(&cur[q]);
        path_free(&nxt[q]);
    }
    free(cur);
    free(nxt);
    free(cand);
    free(lam_i);
    free(tmp);
    free(ch);
    return len;
}

void orc_scl_batch(const float* llr, int64_t B, int N, const uint8_t* frozen, const uint8_t* da,
                   int c, uint32_t poly, int L, int rule, uint8_t* u_hat, uint8_t* crc_ok, double* pm) {
    for (int64_t f = 0; f < B; f++)
        orc_scl_frame(llr + f * N, N, frozen, da, c, poly, L, rule, u_hat + f * N, crc_ok + f,
                      pm ? pm + f : NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Hybrid decoder (Sec. III): BP with at most max_iter iterations and the    */
/* early stop of Sec. II-B -- stop 1 the re-encoding check, stop 2 the CRC,   */
/* which the paper allows in its place; if BP does not end with a valid CRC,  */
/* the frame is decoded again by CA-SCL from the channel LLRs.  info_out gets */
/* the K info bits of whichever result is kept.  bp_rule selects the BP       */
/* update rule (0 min-sum, 1 the exact rule of Sec. II-B); the list decoder   */
/* keeps the min-sum metric.                                                  */
/* ------------------------------------------------------------------------ */

void orc_hybrid_batch(const float* llr, int64_t B, int N, const uint8_t* frozen, const uint8_t* da,
                      int K, int c, uint32_t poly, int max_iter, int stop, double llr_max, int bp_rule,
                      const double* W, int L, uint8_t* info_out, uint8_t* used_scl, int32_t* iters) {
    uint8_t* u = (uint8_t*)malloc(N);
    for (int64_t f = 0; f < B; f++) {
        uint8_t ok = 0, cok = 0;
        int it = orc_bp_frame(llr + f * N, N, frozen, c, poly, max_iter, stop, llr_max, bp_rule, W, u,
                              NULL, NULL, &ok, NULL);
        if (iters) iters[f] = it;
        used_scl[f] = (uint8_t)(ok ? 0 : 1);
        if (!ok) orc_scl_frame(llr + f * N, N, frozen, da, c, poly, L, 0, u, &cok, NULL, NULL, NULL);
        int q = 0;
        for (int i = 0; i < N && q < K; i++)
            if (!frozen[i]) info_out[f * K + q++] = u[i];
    }
    free(u);
}

/* ------------------------------------------------------------------------ */
/* Weighted (learned) min-sum BP: loss and its gradient.                     */
/* Not in the paper.  Forward: the weighted BP above, T iterations, no early */
/* stop.  Losses of a frame (times `scale`), with lam_{t,i} = L[0][i] +      */
/* R[0][i] after iteration t and z_{t,i} = (2 u_i - 1) lam_{t,i}:             */
/*   kind 0: sum over the non-frozen i of softplus(z_{T,i}) (binary           */
/*           cross-entropy of P(u_i = 1) = sigmoid(-lam_i) after the last     */
/*           iteration);                                                      */
/*   kind 1: the same sum after every iteration, summed over t;               */
/*   kind 2: prod_t (1 - exp(-S_t)), S_t = sum_i softplus(z_{t,i}): with the  */
/*           bits taken as independent, exp(-S_t) is the probability that    */
/*           every non-frozen decision after iteration t is right, so the     */
/*           product is the probability that no iteration gets the whole     */
/*           frame right -- a smooth stand-in for a BP failure within T       */
/*           iterations (the frames the hybrid hands to the list decoder);    */
/*   kind 3: sum_{u=1}^{T-1} P_u + c P_T, P_u = prod_{t<=u} (1 - exp(-S_t)), */
/*           c = fail_weight: P_u is the probability (same independence)     */
/*           that the frame is still undecided after iteration u, so the sum  */
/*           is the expected number of iterations beyond the first that an   */
/*           early-stopping decoder runs, and c P_T (c times the kind-2 loss) */
/*           prices a frame handed to the list decoder at c iterations.       */
/* Backward (reverse mode, by hand): iterations T..1; inside one, the L sweep */
/* is undone first (s = 0..n-1), then the R sweep (s = n-1..0).  Rules:       */
/*   d clip(p)/dp = 1 if |p| <= LLR_max (inclusive), else 0;                  */
/*   g(a,b) = a sgn(b) when |a| <= |b| (ties go to a), else b sgn(a);         */
/*   the sign factor itself has zero derivative.                              */
/* dW accumulates over frames (in double); dllr (optional) is the gradient    */
/* with respect to the channel LLRs, including the clip at load.              */
/* ------------------------------------------------------------------------ */

static void g_partials(real a, real b, real* da, real* db) {
    if (fabs(a) <= fabs(b)) { *da = sgn(b); *db = 0; }
    else { *da = 0; *db = sgn(a); }
}

/* Adjoint of the weighted BP given dlam = d loss / d lambda (N values; zero on
 * frozen positions): accumulates dW (double) and writes dllr (optional). */
void orc_wbp_backward_frame(const float* llr, int N, const uint8_t* frozen, int T, double llr_max,
                            const double* W, const double* dlam, int dlam_iters, double* dW,
                            double* dllr) {
    int n = ilog2(N);
    real lmax = (real)llr_max;
    size_t per = (size_t)2 * n * N;
    /* forward, saving every message produced */
    double* save = (double*)malloc(sizeof(double) * per * T);
    uint8_t* uh = (uint8_t*)malloc(N);
    uint8_t ok;
    orc_bp_frame(llr, N, frozen, 0, 0, T, 0, llr_max, 0, W, uh, NULL, NULL, &ok, save);
    /* the saved values are exact copies of `real` messages */
    real* Rch = (real*)malloc(sizeof(real) * N);  /* clipped channel */
    real* R0 = (real*)malloc(sizeof(real) * N);   /* frozen prior row */
    for (int i = 0; i < N; i++) {
        Rch[i] = clip((real)llr[i], lmax);
        R0[i] = frozen[i] ? lmax : (real)0;
    }
    /* adjoints of the current message rows */
    real* aL = (real*)calloc((size_t)(n + 1) * N, sizeof(real));
    real* aR = (real*)calloc((size_t)(n + 1) * N, sizeof(real));
#define SAVED_R(t, s, i) ((real)save[(size_t)(t) * per + ((size_t)0 * n + (s)) * N + (i)])
#define SAVED_L(t, s, i) ((real)save[(size_t)(t) * per + ((size_t)1 * n + (s)) * N + (i)])
    /* value of row r of R during iteration t (0-based): row 0 constant, row r >= 1 saved */
#define RV(t, r, i) ((r) == 0 ? R0[i] : SAVED_R(t, (r) - 1, i))
    /* value of row r of L "as of the end of iteration t" (t = -1: initial state) */
#define LV(t, r, i) ((r) == n ? Rch[i] : ((t) < 0 ? (real)0 : SAVED_L(t, r, i)))
    for (int t = T - 1; t >= 0; t--) {
        const double* Wt = W ? W + (size_t)t * per : NULL;
        /* the loss reads LLR(u) after iteration t (every iteration when
         * dlam_iters == T, the last one when it is 1); row 0 of L feeds
         * nothing else, so its adjoint is exactly d loss / d lambda_t */
        if (dlam_iters == T || t == T - 1) {
            const double* dl = dlam + (size_t)(dlam_iters == T ? t : 0) * N;
            for (int i = 0; i < N; i++) aL[0 * N + i] = (real)dl[i];
        }
        /* undo the L sweep: forward order s = n-1..0, reverse s = 0..n-1 */
        for (int s = 0; s < n; s++) {
            int d = 1 << s;
            for (int i = 0; i < N; i++) {
                if (i & d) continue;
                int j = i + d;
                real a1 = LV(t, s + 1, i), a2 = LV(t, s + 1, j);
                real r1 = RV(t, s, i), r2 = RV(t, s, j);
                real wi = Wt ? (real)Wt[(1 * n + s) * N + i] : (real)1;
                real wj = Wt ? (real)Wt[(1 * n + s) * N + j] : (real)1;
                real bi = a2 + r2;
                real gi = g_minsum(a1, bi), gj = g_minsum(r1, a1);
                real pi = wi * gi, pj = FMA(wj, gj, a2);
                real di = (fabs(pi) <= lmax) ? aL[s * N + i] : (real)0;
                real dj = (fabs(pj) <= lmax) ? aL[s * N + j] : (real)0;
                aL[s * N + i] = 0;
                aL[s * N + j] = 0;
                if (dW) {
                    dW[(size_t)t * per + (1 * n + s) * N + i] += (double)(di * gi);
                    dW[(size_t)t * per + (1 * n + s) * N + j] += (double)(dj * gj);
                }
                real ga, gb;
                g_partials(a1, bi, &ga, &gb);
                real ci = di * wi;
                aL[(s + 1) * N + i] += ci * ga;
                aL[(s + 1) * N + j] += ci * gb;
                if (s > 0) aR[s * N + j] += ci * gb;
                g_partials(r1, a1, &ga, &gb);
                real cj = dj * wj;
                if (s > 0) aR[s * N + i] += cj * ga;
                aL[(s + 1) * N + i] += cj * gb;
                aL[(s + 1) * N + j] += dj;
            }
        }
        /* undo the R sweep: forward order s = 0..n-1, reverse s = n-1..0 */
        for (int s = n - 1; s >= 0; s--) {
            int d = 1 << s;
            for (int i = 0; i < N; i++) {
                if (i & d) continue;
                int j = i + d;
                real r1 = RV(t, s, i), r2 = RV(t, s, j);
                real l1 = LV(t - 1, s + 1, i), l2 = LV(t - 1, s + 1, j);
                real wi = Wt ? (real)Wt[(0 * n + s) * N + i] : (real)1;
                real wj = Wt ? (real)Wt[(0 * n + s) * N + j] : (real)1;
                real bi = l2 + r2;
                real gi = g_minsum(r1, bi), gj = g_minsum(r1, l1);
                real pi = wi * gi, pj = FMA(wj, gj, r2);
                real di = (fabs(pi) <= lmax) ? aR[(s + 1) * N + i] : (real)0;
                real dj = (fabs(pj) <= lmax) ? aR[(s + 1) * N + j] : (real)0;
                aR[(s + 1) * N + i] = 0;
                aR[(s + 1) * N + j] = 0;
                if (dW) {
                    dW[(size_t)t * per + (0 * n + s) * N + i] += (double)(di * gi);
                    dW[(size_t)t * per + (0 * n + s) * N + j] += (double)(dj * gj);
                }
                real ga, gb;
                g_partials(r1, bi, &ga, &gb);
                real ci = di * wi;
                if (s > 0) aR[s * N + i] += ci * ga;
                aL[(s + 1) * N + j] += ci * gb;
                if (s > 0) aR[s * N + j] += ci * gb;
                g_partials(r1, l1, &ga, &gb);
                real cj = dj * wj;
                if (s > 0) aR[s * N + i] += cj * ga;
                aL[(s + 1) * N + i] += cj * gb;
                if (s > 0) aR[s * N + j] += dj;
            }
        }
        /* rows 1..n-1 of aL now hold the adjoints of the messages produced in
         * iteration t-1; row n accumulates the channel adjoint across all
         * iterations. */
    }
#undef SAVED_R
#undef SAVED_L
#undef RV
#undef LV
    if (dllr)
        for (int i = 0; i < N; i++)
            dllr[i] = (fabs((real)llr[i]) <= lmax) ? (double)aL[n * N + i] : 0.0;
    free(save);
    free(uh);
    free(Rch);
    free(R0);
    free(aL);
    free(aR);
}

double orc_wbp_grad_frame(const float* llr, int N, const uint8_t* frozen, const uint8_t* u_true,
                          int T, double llr_max, const double* W, double scale, int kind, double fail_weight,
                          double* dW /* [T][2][n][N], accumulated */, double* dllr /* N or NULL */) {
    int n = ilog2(N);
    size_t per = (size_t)2 * n * N;
    uint8_t* uh = (uint8_t*)malloc(N);
    uint8_t ok;
    double* lam = (double*)malloc(sizeof(double) * N);
    int nl = kind ? T : 1;
    double* dlam = (double*)calloc((size_t)nl * N, sizeof(double));
    double* save = kind ? (double*)malloc(sizeof(double) * per * T) : NULL;
    orc_bp_frame(llr, N, frozen, 0, 0, T, 0, llr_max, 0, W, uh, lam, NULL, &ok, save);
    /* lam_{t,i} of the iterations the loss reads */
    double* lt = (double*)malloc(sizeof(double) * (size_t)nl * N);
    for (int q = 0; q < nl; q++) {
        int t = kind ? q : T - 1;
        for (int i = 0; i < N; i++)
            /* LLR(u_i) after iteration t: L row 0 plus the (zero) prior of a
             * non-frozen position, added in working precision as in BP */
            lt[(size_t)q * N + i] = kind ? (double)((real)save[(size_t)t * per + (size_t)n * N + i] + (real)0) : lam[i];
    }
    double loss = 0.0;
    if (kind < 2) {
        for (int q = 0; q < nl; q++)
            for (int i = 0; i < N; i++) {
                if (frozen[i]) continue;
                double sgn_u = u_true[i] ? 1.0 : -1.0;
                double z = sgn_u * lt[(size_t)q * N + i];
                loss += softplus(z);
                /* d softplus(z)/d lam = sgn_u * sigmoid(z) */
                double sig = 1.0 / (1.0 + exp(-z));
                dlam[(size_t)q * N + i] = (double)(real)(scale * sgn_u * sig);
            }
    } else {
        /* S_t, then F = prod_t (1 - e^{-S_t}); dF/dS_t = e^{-S_t} prod_{t' != t} (1 - e^{-S_t'}) */
        double* S = (double*)calloc((size_t)T, sizeof(double));
        for (int t = 0; t < T; t++)
            for (int i = 0; i < N; i++) {
                if (frozen[i]) continue;
                double sgn_u = u_true[i] ? 1.0 : -1.0;
                S[t] += softplus(sgn_u * lt[(size_t)t * N + i]);
            }
        /* q_t = 1 - e^{-S_t}: the probability that iteration t leaves some decision wrong */
        double* q = (double*)malloc(sizeof(double) * T);
        for (int t = 0; t < T; t++) q[t] = -expm1(-S[t]);
        double F = 1.0;
        for (int t = 0; t < T; t++) F *= q[t];
        if (kind == 2) {
            loss = F;
        } else {
            /* sum over u = 1..T-1 (iterations counted from 1) of P_u, plus c P_T */
            loss = 0.0;
            for (int u = 0; u < T - 1; u++) {
                double P = 1.0;
                for (int t = 0; t <= u; t++) P *= q[t];
                loss += P;
            }
            loss += fail_weight * F;
        }
        for (int t = 0; t < T; t++) {
            /* d loss / d S_t: dq_t/dS_t = e^{-S_t}, times every product that holds q_t
               with q_t taken out */
            double dS;
            if (kind == 2) {
                dS = exp(-S[t]);
                for (int t2 = 0; t2 < T; t2++)
                    if (t2 != t) dS *= q[t2];
            } else {
                double acc = 0.0;
                for (int u = t; u < T - 1; u++) {
                    double P = 1.0;
                    for (int t2 = 0; t2 <= u; t2++)
                        if (t2 != t) P *= q[t2];
                    acc += P;
                }
                double PT = 1.0;
                for (int t2 = 0; t2 < T; t2++)
                    if (t2 != t) PT *= q[t2];
                acc += fail_weight * PT;
                dS = exp(-S[t]) * acc;
            }
            for (int i = 0; i < N; i++) {
                if (frozen[i]) continue;
                double sgn_u = u_true[i] ? 1.0 : -1.0;
                double z = sgn_u * lt[(size_t)t * N + i];
                double sig = 1.0 / (1.0 + exp(-z));
                dlam[(size_t)t * N + i] = (double)(real)(scale * dS * sgn_u * sig);
            }
        }
        free(q);
        free(S);
    }
    orc_wbp_backward_frame(llr, N, frozen, T, llr_max, W, dlam, nl, dW, dllr);
    free(uh);
    free(lam);
    free(lt);
    free(dlam);
    free(save);
    return loss * scale;
}

void orc_wbp_backward_batch(const float* llr, int64_t B, int N, const uint8_t* frozen, int T, double llr_max,
                            const double* W, const double* dlam, int dlam_iters, double* dW, double* dllr) {
    for (int64_t f = 0; f < B; f++)
        orc_wbp_backward_frame(llr + f * N, N, frozen, T, llr_max, W, dlam + (size_t)f * dlam_iters * N,
                               dlam_iters, dW, dllr ? dllr + f * N : NULL);
}

double orc_wbp_grad_batch(const float* llr, int64_t B, int N, const uint8_t* frozen,
                          const uint8_t* u_true, int T, double llr_max, const double* W,
                          double scale, int kind, double fail_weight, double* dW, double* dllr) {
    double loss = 0.0;
    for (int64_t f = 0; f < B; f++)
        loss += orc_wbp_grad_frame(llr + f * N, N, frozen, u_true + f * N, T, llr_max, W, scale, kind,
                                   fail_weight, dW, dllr ? dllr + f * N : NULL);
    return loss;
}

/* Adam (Kingma and Ba, 2015) on `count` parameters, step t >= 1. */
void orc_adam_step(double* w, const double* grad, double* m, double* v, int64_t count, int t,
                   double lr, double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t q = 0; q < count; q++) {
        m[q] = beta1 * m[q] + (1.0 - beta1) * grad[q];
        v[q] = beta2 * v[q] + (1.0 - beta2) * grad[q] * grad[q];
        double mh = m[q] / c1, vh = v[q] / c2;
        w[q] -= lr * mh / (sqrt(vh) + eps);
    }
}
