// bp_geom.hpp -- compile-time data layout of the BP kernel (no HIP
// dependencies, so host programs can verify it).
//
// A frame of N = 2^n nodes per stage row is spread over T = N / V threads
// (V = 2^r values per thread).  Window k keeps index bits [wbase(k),
// wbase(k) + r) in registers and processes the PE columns cbeg(k)..cend(k)-1;
// the remaining index bits come from the thread number in increasing order.
// Across a window boundary one row is re-laid out through LDS.  Its LDS word
// address is sum_b bit_b(i) * c_b over the index bits (and frame-slot bits),
// with coefficients whose residues mod 32 make the lanes of each
// half-wavefront hit distinct banks in both layouts and that keep the map
// injective.  Boundaries inside a wavefront take them greedily (each bit the
// smallest coefficient with its residue that keeps the map injective, the
// destination layout's lane bits first), which packs a wavefront's 64 V values
// into little more than 64 V words; boundaries across wavefronts use
// super-increasing coefficients.
#pragma once

namespace polarhip {
namespace bp {

constexpr int kBankBits = 5;
constexpr int kMaxPB = 24;  // pseudo-bits: index bits + frame-slot bits
constexpr int kMaxBnd = 12;

constexpr int kGreedySpan = 4096;  // words of one wavefront's region, at most

// Greedy injective coefficients: bits order[0..no) in turn get the smallest
// c >= 1 with c = resid (mod 32) when resid >= 0 (any c otherwise) such that
// no two bit patterns map to the same word.  Returns the span (words), or a
// value above kGreedySpan when none fits.
constexpr int greedy_coefficients(const int* order, int no, const int* resid, int* coef) {
    bool mem[kGreedySpan] = {};
    int list[1 << 10] = {};
    int nl = 1, maxa = 0;
    mem[0] = true;
    for (int j = 0; j < no; ++j) {
        const int pb = order[j];
        const int step = resid[pb] >= 0 ? 32 : 1;
        int c = resid[pb] >= 0 ? resid[pb] % 32 : 1;
        if (c == 0) c = step;
        for (; c < kGreedySpan; c += step) {
            bool fits = true;
            for (int a = 0; a < nl && fits; ++a) {
                const int x = list[a] + c;
                fits = x < kGreedySpan && !mem[x];
            }
            if (fits) break;
        }
        if (c >= kGreedySpan || 2 * nl > (1 << 10)) return kGreedySpan + 1;
        coef[pb] = c;
        for (int a = 0; a < nl; ++a) {
            const int x = list[a] + c;
            mem[x] = true;
            list[nl + a] = x;
            if (x > maxa) maxa = x;
        }
        nl *= 2;
    }
    return maxa + 1;
}

constexpr int ilog2c(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

struct Boundary {
    int c[kMaxPB];  // LDS word coefficient of each pseudo bit
    int size;       // words spanned
    bool cross;     // layouts differ in which index bits the wave id holds
    int buf_r;      // buffer (word offset) used for R rows crossing this boundary
    int buf_l;      // buffer (word offset) used for L rows
};

struct Table {
    Boundary b[kMaxBnd];
    int words;  // total transpose buffer words
};

template <int NLOG, int RLOG>
struct Geom {
    static constexpr int n = NLOG, r = RLOG, N = 1 << NLOG, V = 1 << RLOG;
    static constexpr int P = n - r;   // thread bits per frame
    static constexpr int T = 1 << P;  // threads per frame
    static constexpr int FPW = T < 64 ? 64 / T : 1;
    static constexpr int SLOTB = ilog2c(FPW);
    static constexpr int WG = T < 64 ? 64 : T;
    static constexpr int NWAVES = WG / 64;
    static constexpr int NWIN = (n + r - 1) / r;
    static constexpr int NB = NWIN - 1;
    static constexpr int NPB = n + SLOTB;
    static constexpr int TL = T < 64 ? T : 64;  // checker lanes of a frame
    static constexpr int CB = N / TL;           // bits per checker lane
    static_assert(r >= 1 && r <= n, "bad register bits");
    static_assert(CB <= 64, "N too large for the check");
    static_assert(NPB <= kMaxPB && NB <= kMaxBnd, "table too small");

    static constexpr int wbase(int k) { return k * r < n - r ? k * r : n - r; }
    static constexpr int cbeg(int k) { return k * r; }
    static constexpr int cend(int k) { return (k + 1) * r < n ? (k + 1) * r : n; }
    // pseudo bit held by thread/lane bit q in window k (q < P: index bit;
    // P <= q < 6: frame-slot bit when several frames share a wavefront)
    static constexpr int tpb(int k, int q) {
        return q < P ? (q < wbase(k) ? q : q + r) : n + (q - P);
    }
    static constexpr bool is_cross(int k) {
        for (int q = 6; q < P; ++q)
            if (tpb(k, q) != tpb(k + 1, q)) return true;
        return false;
    }
    static constexpr bool is_wave_bit(int k, int pb) {
        for (int q = 6; q < P; ++q)
            if (tpb(k, q) == pb || tpb(k + 1, q) == pb) return true;
        return false;
    }

    static constexpr Table make_table() {
        Table t{};
        int ws = 0;  // word stride of one wavefront's region in the shared intra buffer
        for (int k = 0; k < NB; ++k) {
            Boundary& B = t.b[k];
            B.cross = is_cross(k);
            int SA[kBankBits], SB[kBankBits];
            int nh = 0;
            for (int q = 0; q < kBankBits && q < 6; ++q) {
                SA[nh] = tpb(k, q);
                SB[nh] = tpb(k + 1, q);
                ++nh;
            }
            int resid[kMaxPB];
            for (int i = 0; i < kMaxPB; ++i) resid[i] = -1;
            int nres = 0;
            // shared bits first, then the bits that only one layout spreads over
            // lanes, paired with equal residues
            for (int a = 0; a < nh; ++a) {
                bool inB = false;
                for (int b = 0; b < nh; ++b) inB = inB || (SB[b] == SA[a]);
                if (inB) resid[SA[a]] = 1 << nres++;
            }
            int oa[kBankBits], ob[kBankBits], na = 0, nb = 0;
            for (int a = 0; a < nh; ++a) {
                bool inB = false;
                for (int b = 0; b < nh; ++b) inB = inB || (SB[b] == SA[a]);
                if (!inB) oa[na++] = SA[a];
            }
            for (int b = 0; b < nh; ++b) {
                bool inA = false;
                for (int a = 0; a < nh; ++a) inA = inA || (SA[a] == SB[b]);
                if (!inA) ob[nb++] = SB[b];
            }
            for (int j = 0; j < na; ++j) {
                resid[oa[j]] = 1 << nres;
                resid[ob[j]] = 1 << nres;
                ++nres;
            }
            // assignment order: residue-constrained bits by residue, then the
            // free bits, wave bits last (intra boundaries)
            int order[kMaxPB], no = 0;
            for (int q = 0; q < nres; ++q)
                for (int pb = 0; pb < NPB; ++pb)
                    if (resid[pb] == (1 << q)) order[no++] = pb;
            for (int pb = 0; pb < NPB; ++pb)
                if (resid[pb] < 0 && !is_wave_bit(k, pb)) order[no++] = pb;
            int S = 0;
            if (!B.cross) {
                // destination layout's lane bits first, then the rest
                int og[kMaxPB], ng = 0;
                bool used[kMaxPB] = {};
                for (int j = 0; j < no; ++j) {
                    bool lane_b = false;
                    for (int q = 0; q < 6; ++q) lane_b = lane_b || (tpb(k + 1, q) == order[j]);
                    if (lane_b) {
                        og[ng++] = order[j];
                        used[order[j]] = true;
                    }
                }
                for (int j = 0; j < no; ++j)
                    if (!used[order[j]]) og[ng++] = order[j];
                S = greedy_coefficients(og, ng, resid, B.c) - 1;
            } else {
                for (int j = 0; j < no; ++j) {
                    int pb = order[j];
                    int c = S + 1;
                    if (resid[pb] >= 0) {
                        int m = 1 << kBankBits;
                        while (c % m != resid[pb] % m) ++c;
                    }
                    B.c[pb] = c;
                    S += c;
                }
            }
            B.size = S + 1;
            if (!B.cross && S + 1 > ws) ws = S + 1;
            // wave bits of a cross boundary: plain super-increasing continuation
            if (B.cross) {
                for (int pb = 0; pb < NPB; ++pb)
                    if (resid[pb] < 0 && is_wave_bit(k, pb)) {
                        B.c[pb] = S + 1;
                        S += S + 1;
                    }
                B.size = S + 1;
            }
        }
        // intra boundaries share one buffer; each wavefront owns a stride ws
        int off = 0;
        int intra_words = 0;
        for (int k = 0; k < NB; ++k) {
            Boundary& B = t.b[k];
            if (B.cross) continue;
            int j = 0;
            for (int q = 6; q < P; ++q) {
                B.c[tpb(k, q)] = ws << j;
                ++j;
            }
            B.size = ws << j;
            if (B.size > intra_words) intra_words = B.size;
            B.buf_r = 0;
            B.buf_l = 0;
        }
        off = intra_words;
        for (int k = 0; k < NB; ++k) {
            Boundary& B = t.b[k];
            if (!B.cross) continue;
            B.buf_r = off;
            off += B.size;
            B.buf_l = off;
            off += B.size;
        }
        t.words = off > 0 ? off : 1;
        return t;
    }
    static constexpr Table TAB = make_table();
    static_assert(TAB.words > 0, "layout table");

    // register part of the LDS word address of value v in window k at boundary j
    static constexpr int reg_off(int j, int k, int v) {
        int o = 0;
        for (int q = 0; q < r; ++q)
            if ((v >> q) & 1) o += TAB.b[j].c[wbase(k) + q];
        return o;
    }
};

// node index held by thread t, register v, in window k
template <class G>
constexpr int node_index(int k, int t, int v) {
    const int b = G::wbase(k);
    return (t & ((1 << b) - 1)) | (v << b) | ((t >> b) << (b + G::r));
}

// LDS word (within the transpose buffers) of thread t / frame slot `slot`,
// register v, layout of window k, boundary j, row direction (R or L)
template <class G>
constexpr int lds_word(int j, int k, int t, int slot, int v, bool is_r) {
    int a = is_r ? G::TAB.b[j].buf_r : G::TAB.b[j].buf_l;
    for (int q = 0; q < G::P; ++q)
        if ((t >> q) & 1) a += G::TAB.b[j].c[G::tpb(k, q)];
    for (int q = 0; q < G::SLOTB; ++q)
        if ((slot >> q) & 1) a += G::TAB.b[j].c[G::n + q];
    return a + G::reg_off(j, k, v);
}

}  // namespace bp
}  // namespace polarhip
