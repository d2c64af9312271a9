// bp.hip -- batched min-sum belief-propagation decoder of polar codes
// (Sec. II-B, Fig. 2), plain and weighted, with early stopping by the
// re-encoding check or the CRC.
//
// Design (MI355X / gfx950).  Messages live in registers.  A frame of N = 2^n
// nodes per stage is spread over T = N / V threads, each holding V = 2^r nodes
// of every stage row.  Which r index bits a thread holds in registers changes
// along the sweep: window k keeps bits [b_k, b_k + r) in registers and handles
// the PE columns that pair those bits, so every butterfly is computed inside
// one thread without communication.  Between windows the single row on the
// boundary is re-laid out through LDS (one write and one read per value).
// The LDS address of an index is a sum of per-bit coefficients chosen at
// compile time so that, for both layouts of a boundary, the 32 lanes of a
// half-wavefront hit 32 different banks and the register part of the address
// is an immediate offset.  Boundaries whose layouts differ only inside one
// wavefront need no barrier; the others are separated by a workgroup barrier.
// When a frame needs fewer than 64 threads, one wavefront carries 64 / T
// frames, each leaving the iteration loop on its own.
//
// PE arithmetic (min-sum inference): a PE's two g terms share one operand a,
// and g(a, b) = sgn(a) clamp(b, -|a|, |a|), so the sign of a is moved once
// into the weight and each g is one clamp; with one weight per stage column
// and every weight within [-1, 1] a second copy of the decoder leaves out the
// first output's clip, which cannot act there.
//
// Early stop (Sec. II-B): after each iteration the hard decisions on LLR(u)
// and LLR(x) are stored as bits (eight-register layouts; bytes otherwise) and
// gathered into words of N / 64 bits per checker lane, u_hat is re-encoded
// with shifts inside words and lane exchanges across words, and compared with
// x_hat; the CRC test uses per-nibble syndrome tables.
#include "bp_common.hpp"

namespace polarhip {
namespace bp {

template <class G>
__device__ __forceinline__ uint64_t load_bits(const uint8_t* src) {
    // CB bytes (0/1) starting at src -> CB-bit word, bit j = byte j
    uint64_t w = 0;
    if constexpr (G::CB >= 4) {
#pragma unroll
        for (int q = 0; q < G::CB / 4; ++q) {
            uint32_t d = reinterpret_cast<const uint32_t*>(src)[q];
            uint32_t nib = ((d * 0x01020408u) >> 24) & 0xFu;
            w |= (uint64_t)nib << (4 * q);
        }
    } else {
#pragma unroll
        for (int q = 0; q < G::CB; ++q) w |= (uint64_t)(src[q] & 1u) << q;
    }
    return w;
}

// Packed decisions (V = 8 and a frame of at least one wavefront): bit j of
// the frame's bit array is node j.  Checker lane l's CB consecutive bits, read
// in one access.
template <class G>
__device__ __forceinline__ uint64_t read_bits(const uint8_t* bits, int lane) {
    if constexpr (G::CB == 8) return bits[lane];
    else if constexpr (G::CB == 16) return reinterpret_cast<const uint16_t*>(bits)[lane];
    else if constexpr (G::CB == 32) return reinterpret_cast<const uint32_t*>(bits)[lane];
    else return reinterpret_cast<const uint64_t*>(bits)[lane];
}

template <class G, bool PACKED>
__device__ __forceinline__ uint64_t lane_bits(const uint8_t* src, int lane) {
    if constexpr (PACKED) return read_bits<G>(src, lane);
    else return load_bits<G>(src + lane * G::CB);
}

// Lane exchanges of the stop tests, all in VALU (no LDS round trip, which
// the early-stop test would otherwise wait on in every iteration):
// lane ^ 1, ^ 2 by quad permutes; a lane of the other quad of its eight, the
// other half of its row of sixteen by the half-row and row mirrors (for a
// reduction any lane of the other half serves); lane ^ 16, ^ 32 by the gfx950
// row swaps.
// lane permutation CTRL of v (a full permutation of each row: every lane is
// written); the zero "old" value lets the compiler fold the move into the XOR
// that takes it
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// XOR of s over each group of TL consecutive lanes (TL a power of two <= 64);
// every lane of the group gets it
template <int TL>
__device__ __forceinline__ uint32_t group_xor(uint32_t s) {
    if constexpr (TL > 1) s ^= dpp32<0xB1>(s);   // quad_perm [1,0,3,2]
    if constexpr (TL > 2) s ^= dpp32<0x4E>(s);   // quad_perm [2,3,0,1]
    if constexpr (TL > 4) s ^= dpp32<0x141>(s);  // row_half_mirror
    if constexpr (TL > 8) s ^= dpp32<0x140>(s);  // row_mirror
    if constexpr (TL > 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(s, s, false, false);
        s = r[0] ^ r[1];
    }
    if constexpr (TL > 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(s, s, false, false);
        s = r[0] ^ r[1];
    }
    return s;
}

// the value of lane + Q (Q a power of two <= 32) for the lanes whose bit Q is
// clear; what the other lanes get is not used.  Row shifts inside a row of
// sixteen; for 16 and 32 the row swaps, whose second result holds, on those
// lanes, the partner row
template <int Q>
__device__ __forceinline__ uint32_t from_lane_above(uint32_t v) {
    if constexpr (Q < 16) {
        // row_shl: lane i reads lane i + Q of its row (lanes past the row's end get 0)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + Q, 0xF, 0xF, false);
    } else if constexpr (Q == 16) {
        return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    } else {
        static_assert(Q == 32, "distance");
        return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    }
}

// bits p of a 64-bit word with p & d == 0 (d a power of two)
constexpr uint64_t low_half_mask(int d) {
    uint64_t m = 0;
    for (int p = 0; p < 64; ++p)
        if ((p & d) == 0) m |= 1ull << p;
    return m;
}

// u G == x on the packed words of one frame; every checker lane gets the answer
template <class G, bool PACKED>
__device__ __forceinline__ bool reencode_check(const uint8_t* ub, const uint8_t* xb, int lane) {
    uint64_t u = lane_bits<G, PACKED>(ub, lane);
    uint64_t x = lane_bits<G, PACKED>(xb, lane);
    // butterflies inside a word: distances 1, 2, .. CB/2 (masks fixed at compile time)
    static_for<0, 6>([&](auto D) {
        constexpr int d = 1 << decltype(D)::value;
        if constexpr (d < G::CB) {
            constexpr uint64_t m = low_half_mask(d);
            u ^= (u >> d) & m;
        }
    });
    // butterflies across the checker lanes: lanes with bit q clear take lane + q
    static_for<0, 6>([&](auto QC) {
        constexpr int q = 1 << decltype(QC)::value;
        if constexpr (q < G::TL) {
            const uint32_t lo = from_lane_above<q>((uint32_t)u);
            const uint32_t hi = G::CB > 32 ? from_lane_above<q>((uint32_t)(u >> 32)) : 0u;
            if ((lane & q) == 0) u ^= ((uint64_t)hi << 32) | lo;
        }
    });
    uint64_t bad = __ballot(u != x);
    if constexpr (G::TL < 64) {
        const int grp = (__lane_id() / G::TL) * G::TL;
        bad = (bad >> grp) & ((1ull << G::TL) - 1ull);
    }
    return bad == 0;
}

template <class G, bool PACKED>
__device__ __forceinline__ bool crc_check(const CodeDev& code, const uint8_t* ub, int lane) {
    if (code.c == 0) return true;
    uint64_t u = lane_bits<G, PACKED>(ub, lane);
    uint32_t s = 0;
    const uint32_t* tab = code.syn_nib + (size_t)(lane * G::CB / 4) * 16;
    if constexpr (G::CB >= 4) {
#pragma unroll
        for (int g = 0; g < G::CB / 4; ++g) s ^= tab[g * 16 + ((u >> (4 * g)) & 0xF)];
    } else {
        // fewer than 4 bits per lane: take the nibble from the lanes of the group
        const int g = lane * G::CB / 4;
        const int sh = (lane * G::CB) & 3;
        uint32_t part = (uint32_t)(u << sh);
        uint32_t nib = part;
#pragma unroll
        for (int q = 1; q < 4 / G::CB; ++q) nib |= __shfl_xor(part, q, 64);
        s = (sh == 0) ? code.syn_nib[(size_t)g * 16 + (nib & 0xF)] : 0u;
    }
    return group_xor<G::TL>(s) == 0;
}

// LDS of one workgroup: transpose buffers, the packed-decision staging and
// the wavefronts' partial CRC syndromes (two sets, taken by iteration parity)
template <class G>
struct BpShared {
    float tb[G::TAB.words];
    __attribute__((aligned(16))) uint8_t ubytes[G::FPW * G::N];
    __attribute__((aligned(16))) uint8_t xbytes[G::FPW * G::N];
    uint32_t syn[2][G::NWAVES];
};

// CRC test of a frame of at least one wavefront whose thread t holds its own
// packed decisions, nodes 8t .. 8t + 7 (nibble positions 2t and 2t + 1): each
// thread XORs the syndromes of its two nibbles, each wavefront reduces its
// lanes, and the frame's wavefronts combine their words through LDS.  syn is
// one of two sets taken by iteration parity: a wavefront's next write goes to
// the other set, and the one after it follows the next test's barrier, which
// every wavefront reaches only after its reads.  Every thread of the frame gets
// the answer; ends with a frame-wide barrier.
template <class G>
__device__ __forceinline__ bool crc_check_own(const CodeDev& code, uint32_t bits, int t, uint32_t* syn) {
    static_assert(G::V == 8 && G::T >= 64, "packed decisions of whole wavefronts");
    uint32_t s = 0;
    if (code.c != 0) {
        // byte offsets of the two table entries (bits < 256) from the
        // table's uniform base: 32-bit lane offsets, no per-lane pointer
        const uint8_t* tab = reinterpret_cast<const uint8_t*>(code.syn_nib);
        const uint32_t row = (uint32_t)t << 7;
        const uint32_t o0 = row | ((bits & 15u) << 2);
        const uint32_t o1 = row | 64u | ((bits >> 2) & 0x3Cu);
        s = group_xor<64>(*reinterpret_cast<const uint32_t*>(tab + o0) ^
                          *reinterpret_cast<const uint32_t*>(tab + o1));
    }
    if constexpr (G::NWAVES == 1) {
        frame_sync<G>();
        return s == 0;
    } else {
        if ((t & 63) == 0) syn[t >> 6] = s;
        frame_sync<G>();
        uint32_t a = 0;
#pragma unroll
        for (int w = 0; w < G::NWAVES; ++w) a ^= syn[w];
        return a == 0;
    }
}

// Where one frame's data lives.  SAVE (training): every message a column
// produces is also written to sv[iteration][direction][column][node],
// direction 0 = R (row s+1 of column s), 1 = L (row s), for the adjoint kernel.
struct FrameIO {
    const float* llr;   // [N] channel LLRs
    uint8_t* u_hat;     // [N] or null
    uint8_t* info;      // [K] or null: information bits, written when the verdict is ok
    float* llr_u;       // [N] or null
    int32_t* iters;     // one value or null
    uint8_t* ok;        // one value or null
    float* saved;       // SAVE only
};

// Decode one frame: thread t of the frame's T threads, frame slot `slot` of
// its wavefront (T < 64) or workgroup.  Returns the verdict (for queues).
// NOCLIP (per-stage weights, every weight within [-1, 1]): the first output
// of a PE is w g with |w g| <= |g| <= lmax, so its clip would return its input
// and is left out.
template <class G, bool WEIGHTED, bool SAVE, int RULE = 0, bool WSTAGE = false, bool NOCLIP = false>
__device__ __forceinline__ bool bp_frame(const CodeDev& code, const FrameIO& io, int max_iter, int stop, float lmax,
                                         const float* __restrict__ W, BpShared<G>& sh, int t, int slot) {
    constexpr int n = G::n, N = G::N, V = G::V, KL = G::NWIN - 1;
    // min-sum inference takes the sign-transfer form of g; training (SAVE)
    // and the exact rule keep the direct form
    constexpr bool FAST = RULE == 0 && !SAVE;
    // decisions stored as bits instead of one byte each (u: one byte per
    // thread of window 0, its eight consecutive nodes; x: one ballot per
    // register and wavefront, since in the last window a wavefront's lanes
    // hold 64 consecutive nodes)
    constexpr bool BITPACK = G::V == 8 && G::T >= 64;
    float* tb = sh.tb;
    const int lane = (G::T < 64) ? t : (lid_x() & 63);
    uint8_t* ub = sh.ubytes + slot * N;
    uint8_t* xb = sh.xbytes + slot * N;

    // LDS bases of this thread for each boundary, on both sides
    int bfrom[G::NB > 0 ? G::NB : 1], bto[G::NB > 0 ? G::NB : 1];
    static_for<0, G::NB>([&](auto J) {
        constexpr int j = decltype(J)::value;
        bfrom[j] = lds_base<G, j, j>(t, slot);
        bto[j] = lds_base<G, j, j + 1>(t, slot);
    });

    // messages: row rho of L / R, each V values in the layout of the window
    // that stores it
    float Lm[n + 1][V];
    float Rm[n + 1][V];
    float prior[V];
#pragma unroll
    for (int s = 0; s <= n; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            Lm[s][v] = 0.0f;
            Rm[s][v] = 0.0f;
        }
    const float* fl = io.llr;
    {
        const int ib = idx_base<G, KL>(t);
#pragma unroll
        for (int v = 0; v < V; ++v) Lm[n][v] = clipf(fl[ib + (v << G::wbase(KL))], lmax);
    }
    uint32_t fmask = 0;  // frozen flags of this thread's nodes in window 0
    {
        const int ib = idx_base<G, 0>(t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            int i = ib + v;
            uint32_t f = (code.frozen_bits[i >> 5] >> (i & 31)) & 1u;
            fmask |= f << v;
            prior[v] = f ? lmax : 0.0f;
        }
    }

    int it = 0;
    bool gok = false, cok = false;
    uint32_t ubits = 0;  // packed decisions of this thread's nodes (BITPACK)
    while (true) {
        const float* Wit = WEIGHTED ? W + (size_t)it * 2 * n * (WSTAGE ? 1 : N) : nullptr;
        float* Sit = SAVE ? io.saved + (size_t)it * 2 * n * N : nullptr;
        // ---------------- R sweep: columns 0..n-1
        static_for<0, G::NWIN>([&](auto KC) {
            constexpr int k = decltype(KC)::value;
            const int ib = idx_base<G, k>(t);
            static_for<G::cbeg(k), G::cend(k)>([&](auto SC) {
                constexpr int s = decltype(SC)::value;
                constexpr int q = s - G::wbase(k);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v & (1 << q)) continue;
                    const int v2 = v | (1 << q);
                    const float r1 = (s == 0) ? prior[v] : Rm[s][v];
                    const float r2 = (s == 0) ? prior[v2] : Rm[s][v2];
                    const float l1 = Lm[s + 1][v], l2 = Lm[s + 1][v2];
                    if constexpr (FAST) {
                        // both g terms share r1: its sign rides on the weight
                        const float x = l2 + r2;
                        if constexpr (WEIGHTED) {
                            float wi, wj;
                            if constexpr (WSTAGE) {
                                wi = wj = Wit[0 * n + s];
                            } else {
                                const float* w = Wit + (size_t)(0 * n + s) * N + ib;
                                wi = w[v << G::wbase(k)];
                                wj = w[v2 << G::wbase(k)];
                            }
                            // column 0: r1 is the prior, 0 or lmax > 0, whose
                            // sign leaves the weight as it is
                            const float si = (s == 0) ? wi : sign_to(wi, r1);
                            const float sj = WSTAGE ? si : ((s == 0) ? wj : sign_to(wj, r1));
                            const float yi = si * clamp_mag(x, r1);
                            Rm[s + 1][v] = NOCLIP ? yi : clipf(yi, lmax);
                            Rm[s + 1][v2] = clipf(__fmaf_rn(sj, clamp_mag(l1, r1), r2), lmax);
                        } else {
                            const float si = (s == 0) ? 1.0f : sign_to(1.0f, r1);
                            Rm[s + 1][v] = si * clamp_mag(x, r1);  // |g| <= |r1| <= lmax
                            Rm[s + 1][v2] = clipf(__fmaf_rn(si, clamp_mag(l1, r1), r2), lmax);
                        }
                        continue;
                    }
                    const float gi = g_rule<RULE>(r1, l2 + r2);
                    const float gj = g_rule<RULE>(r1, l1);
                    if constexpr (WEIGHTED) {
                        float wi, wj;
                        if constexpr (WSTAGE) {
                            wi = wj = Wit[0 * n + s];  // uniform: one scalar load
                        } else {
                            const float* w = Wit + (size_t)(0 * n + s) * N + ib;
                            wi = w[v << G::wbase(k)];
                            wj = w[v2 << G::wbase(k)];
                        }
                        Rm[s + 1][v] = clipf(wi * gi, lmax);
                        Rm[s + 1][v2] = clipf(__fmaf_rn(wj, gj, r2), lmax);
                        if constexpr (SAVE) {
                            float* sv = Sit + (size_t)(0 * n + s) * N + ib;
                            sv[v << G::wbase(k)] = Rm[s + 1][v];
                            sv[v2 << G::wbase(k)] = Rm[s + 1][v2];
                        }
                    } else {
                        // min-sum: |g| <= |r1| <= lmax, so the clip is exact
                        Rm[s + 1][v] = RULE == 0 ? gi : clipf(gi, lmax);
                        Rm[s + 1][v2] = clipf(gj + r2, lmax);
                    }
                }
            });
            if constexpr (k < G::NWIN - 1) {
                transpose_row<G, k, k, k + 1, true>(Rm[G::cend(k)], tb, bfrom[k], bto[k]);
            }
        });
        if (stop != 2) {
            if constexpr (BITPACK) {
                // thread t holds node t + (v << P): the wavefront's ballot for
                // register v is 64-bit word (v << (P - 6)) + w of the array
                uint64_t m[V];
#pragma unroll
                for (int v = 0; v < V; ++v) m[v] = __ballot((Lm[n][v] + Rm[n][v]) < 0.0f);
                if (lane == 0) {
                    uint64_t* xw = reinterpret_cast<uint64_t*>(xb) + (t >> 6);
#pragma unroll
                    for (int v = 0; v < V; ++v) xw[v << (G::P - 6)] = m[v];
                }
            } else {
                const int ib = idx_base<G, KL>(t);
#pragma unroll
                for (int v = 0; v < V; ++v) xb[ib + (v << G::wbase(KL))] = (Lm[n][v] + Rm[n][v]) < 0.0f ? 1 : 0;
            }
        }
        // ---------------- L sweep: columns n-1..0
        static_for_rev<0, G::NWIN>([&](auto KC) {
            constexpr int k = decltype(KC)::value;
            const int ib = idx_base<G, k>(t);
            static_for_rev<G::cbeg(k), G::cend(k)>([&](auto SC) {
                constexpr int s = decltype(SC)::value;
                constexpr int q = s - G::wbase(k);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v & (1 << q)) continue;
                    const int v2 = v | (1 << q);
                    const float r1 = (s == 0) ? prior[v] : Rm[s][v];
                    const float r2 = (s == 0) ? prior[v2] : Rm[s][v2];
                    const float l1 = Lm[s + 1][v], l2 = Lm[s + 1][v2];
                    if constexpr (FAST) {
                        // both g terms share l1
                        const float x = l2 + r2;
                        if constexpr (WEIGHTED) {
                            float wi, wj;
                            if constexpr (WSTAGE) {
                                wi = wj = Wit[1 * n + s];
                            } else {
                                const float* w = Wit + (size_t)(1 * n + s) * N + ib;
                                wi = w[v << G::wbase(k)];
                                wj = w[v2 << G::wbase(k)];
                            }
                            const float si = sign_to(wi, l1);
                            const float sj = WSTAGE ? si : sign_to(wj, l1);
                            const float yi = si * clamp_mag(x, l1);
                            Lm[s][v] = NOCLIP ? yi : clipf(yi, lmax);
                            Lm[s][v2] = clipf(__fmaf_rn(sj, clamp_mag(r1, l1), l2), lmax);
                        } else {
                            const float si = sign_to(1.0f, l1);
                            Lm[s][v] = si * clamp_mag(x, l1);  // |g| <= |l1| <= lmax
                            Lm[s][v2] = clipf(__fmaf_rn(si, clamp_mag(r1, l1), l2), lmax);
                        }
                        continue;
                    }
                    const float gi = g_rule<RULE>(l1, l2 + r2);
                    const float gj = g_rule<RULE>(r1, l1);
                    if constexpr (WEIGHTED) {
                        float wi, wj;
                        if constexpr (WSTAGE) {
                            wi = wj = Wit[1 * n + s];
                        } else {
                            const float* w = Wit + (size_t)(1 * n + s) * N + ib;
                            wi = w[v << G::wbase(k)];
                            wj = w[v2 << G::wbase(k)];
                        }
                        Lm[s][v] = clipf(wi * gi, lmax);
                        Lm[s][v2] = clipf(__fmaf_rn(wj, gj, l2), lmax);
                        if constexpr (SAVE) {
                            float* sv = Sit + (size_t)(1 * n + s) * N + ib;
                            sv[v << G::wbase(k)] = Lm[s][v];
                            sv[v2 << G::wbase(k)] = Lm[s][v2];
                        }
                    } else {
                        Lm[s][v] = RULE == 0 ? gi : clipf(gi, lmax);  // min-sum: |g| <= |l1| <= lmax
                        Lm[s][v2] = clipf(gj + l2, lmax);
                    }
                }
            });
            if constexpr (k > 0) {
                transpose_row<G, k - 1, k, k - 1, false>(Lm[G::cbeg(k)], tb, bto[k - 1], bfrom[k - 1]);
            }
        });
        // ---------------- decisions in window 0 (register bits are the low bits)
        if constexpr (BITPACK) {
            // nodes 8t .. 8t + 7: byte t of the bit array.  LLR(u) = L + prior
            // is never -0 (the prior is +0 or lmax > 0, and a sum of zeros of
            // opposite signs rounds to +0), so its sign bit is the test
            // LLR(u) < 0; each bit is shifted in from the sign (one funnel
            // shift), frozen nodes are cleared after
            ubits = 0;
#pragma unroll
            for (int v = V - 1; v >= 0; --v)
                ubits = __builtin_amdgcn_alignbit(ubits, __float_as_uint(Lm[0][v] + prior[v]), 31);
            ubits &= ~fmask;
            // the CRC stop tests every thread's own bits and stores them once,
            // after the loop
            if (stop != 2) ub[t] = (uint8_t)ubits;
        } else {
            uint64_t pack = 0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float lu = Lm[0][v] + prior[v];
                const uint64_t bit = (((fmask >> v) & 1u) == 0 && lu < 0.0f) ? 1ull : 0ull;
                pack |= bit << (8 * v);
            }
            uint8_t* dst = ub + idx_base<G, 0>(t);
            if constexpr (V == 8) {
                *reinterpret_cast<uint64_t*>(dst) = pack;
            } else if constexpr (V == 4) {
                *reinterpret_cast<uint32_t*>(dst) = (uint32_t)pack;
            } else if constexpr (V == 2) {
                *reinterpret_cast<uint16_t*>(dst) = (uint16_t)pack;
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) dst[v] = (uint8_t)(pack >> (8 * v));
            }
        }
        ++it;
        const bool last = it >= max_iter;
        if (stop == 1) {
            frame_sync<G>();
            gok = reencode_check<G, BITPACK>(ub, xb, lane);
            if (gok || last) {
                cok = crc_check<G, BITPACK>(code, ub, lane);
                break;
            }
        } else if (stop == 2) {
            if constexpr (BITPACK) {
                cok = crc_check_own<G>(code, ubits, t, sh.syn[it & 1]);
            } else {
                frame_sync<G>();
                cok = crc_check<G, BITPACK>(code, ub, lane);
            }
            if (cok || last) break;
        } else if (last) {
            frame_sync<G>();
            gok = reencode_check<G, BITPACK>(ub, xb, lane);
            cok = crc_check<G, BITPACK>(code, ub, lane);
            break;
        }
    }

    // ---------------- outputs (window 0 layout: V consecutive nodes per thread)
    const bool okv = stop == 2 ? cok : (gok && cok);
    {
        const int ib = idx_base<G, 0>(t);
        if (io.u_hat) {
            uint8_t* uo = io.u_hat + ib;
            if constexpr (BITPACK) {
                // ubits: the last iteration's decisions
                uint64_t bytes = 0;
#pragma unroll
                for (int v = 0; v < V; ++v) bytes |= (uint64_t)((ubits >> v) & 1u) << (8 * v);
                *reinterpret_cast<uint64_t*>(uo) = bytes;
            } else {
                const uint8_t* src = ub + ib;
#pragma unroll
                for (int v = 0; v < V; ++v) uo[v] = src[v];
            }
        }
        if (io.llr_u) {
            float* lo = io.llr_u + ib;
#pragma unroll
            // row 0 still holds the last iteration's L messages (the loop
            // leaves right after the decisions that read it)
            for (int v = 0; v < V; ++v) lo[v] = Lm[0][v] + prior[v];
        }
        if constexpr (BITPACK) {
            if (stop == 2 && io.info && okv) {
                // the CRC stop left the bits in registers (frame-uniform branch)
                ub[t] = (uint8_t)ubits;
                frame_sync<G>();
            }
        }
        if (io.info && okv) {
            // the hybrid keeps BP's result: its information bits go out here
            for (int q = t; q < code.K; q += G::T) {
                const int pos = code.info_pos[q];
                io.info[q] = BITPACK ? (uint8_t)((ub[pos >> 3] >> (pos & 7)) & 1u) : ub[pos];
            }
        }
        if (t == 0) {
            if (io.iters) *io.iters = it;
            if (io.ok) *io.ok = (uint8_t)okv;
        }
    }
    return okv;
}

// PERSIST: a grid smaller than the batch walks it (frame slots advance by the
// grid size), so a capped grid leaves room on every CU for other kernels.
// The N = 1024 inference kernel with one weight per stage column (128
// threads per frame) fits 128 VGPRs without spilling inside its loop, which
// lets four waves share a SIMD instead of three.
template <int NLOG, int RLOG, bool WEIGHTED, bool SAVE, bool WSTAGE, bool PERSIST>
constexpr int bp_waves_per_eu() {
    return (NLOG == 10 && RLOG == 3 && WEIGHTED && WSTAGE && !SAVE && !PERSIST) ? 4 : 1;
}

template <int NLOG, int RLOG, bool WEIGHTED, bool SAVE, int RULE = 0, bool WSTAGE = false, bool PERSIST = false>
__global__ __launch_bounds__((Geom<NLOG, RLOG>::WG))
__attribute__((amdgpu_waves_per_eu(bp_waves_per_eu<NLOG, RLOG, WEIGHTED, SAVE, WSTAGE, PERSIST>()))) void bp_kernel(
    CodeDev code, const float* __restrict__ llr, int64_t B, int max_iter, int stop, float lmax,
    const float* __restrict__ W, uint8_t* __restrict__ u_hat, uint8_t* __restrict__ info_out,
    float* __restrict__ llr_u, int32_t* __restrict__ iters_out, uint8_t* __restrict__ ok_out,
    float* __restrict__ saved) {
    using G = Geom<NLOG, RLOG>;
    constexpr int N = G::N;
    __shared__ BpShared<G> sh;
    const int tid = lid_x();
    const int t = (G::T < 64) ? (tid & (G::T - 1)) : tid;
    const int slot = (G::T < 64) ? (tid >> G::P) : 0;
    const int64_t stride = PERSIST ? num_groups_x() * G::FPW : 0;
    // per-stage weights all within [-1, 1]: the clip-free form applies (every
    // wavefront reads the max_iter * 2n weights, which sit in the caches)
    bool unit = false;
    if constexpr (WEIGHTED && WSTAGE && RULE == 0 && !SAVE) {
        float m = 0.0f;
        for (int i = tid & 63; i < max_iter * 2 * G::n; i += 64) m = fmaxf(m, fabsf(W[i]));
        unit = wave_max(m) <= 1.0f;
    }
    for (int64_t f0 = gid_x() * G::FPW; f0 < B; f0 += stride) {
        const int64_t frame = f0 + slot;
        if (PERSIST && G::T >= 64 && f0 != gid_x() * G::FPW) __syncthreads();  // staging reuse
        if (G::T < 64 && frame >= B) return;  // lone wavefront: no barriers to honour
        FrameIO io;
        io.llr = llr + frame * N;
        io.u_hat = u_hat ? u_hat + frame * N : nullptr;
        io.info = info_out ? info_out + frame * code.K : nullptr;
        io.llr_u = llr_u ? llr_u + frame * N : nullptr;
        io.iters = iters_out ? iters_out + frame : nullptr;
        io.ok = ok_out ? ok_out + frame : nullptr;
        io.saved = SAVE ? saved + (size_t)frame * max_iter * 2 * G::n * N : nullptr;
        if constexpr (WEIGHTED && WSTAGE && RULE == 0 && !SAVE) {
            if (unit) bp_frame<G, true, false, 0, true, true>(code, io, max_iter, stop, lmax, W, sh, t, slot);
            else bp_frame<G, true, false, 0, true, false>(code, io, max_iter, stop, lmax, W, sh, t, slot);
        } else {
            bp_frame<G, WEIGHTED, SAVE, RULE, WSTAGE>(code, io, max_iter, stop, lmax, W, sh, t, slot);
        }
        if (!PERSIST) break;
    }
}

// Persistent form for ragged batches: workgroups walk the list ids[0..*count)
// (the count lives on the device); frame id's LLR row starts at element
// io->off[id] of io->llr, its u_hat row at id * u_stride; iters and ok are
// indexed by id; failed frames are appended to fail_ids (one atomic each).
// With io->codes, frame id uses the code io->codes[io->code_of[id]] (all of
// the kernel's block length).
// The unweighted N = 2048 gather kernel (256 threads per frame) fits three
// waves per SIMD instead of two without spilling: its failing frames run every iteration, so more frames in
// flight shorten the mixed batch's longest chain.
template <int NLOG, int RLOG, bool WEIGHTED>
constexpr int gather_waves_per_eu() { return (NLOG == 11 && RLOG == 3 && !WEIGHTED) ? 3 : 1; }

template <int NLOG, int RLOG, bool WEIGHTED>
__global__ __launch_bounds__((Geom<NLOG, RLOG>::WG))
__attribute__((amdgpu_waves_per_eu(gather_waves_per_eu<NLOG, RLOG, WEIGHTED>()))) void bp_gather_kernel(
    CodeDev code, const MixedIo* __restrict__ mio, const int32_t* __restrict__ ids, const int32_t* __restrict__ count,
    int max_iter, int stop, float lmax, const float* __restrict__ W, uint8_t* __restrict__ u_hat, int64_t u_stride,
    int32_t* __restrict__ iters_out, uint8_t* __restrict__ ok_out, int32_t* __restrict__ fail_ids,
    int32_t* __restrict__ fail_count) {
    using G = Geom<NLOG, RLOG>;
    __shared__ BpShared<G> sh;
    const int tid = lid_x();
    const int t = (G::T < 64) ? (tid & (G::T - 1)) : tid;
    const int slot = (G::T < 64) ? (tid >> G::P) : 0;
    const int64_t cnt = *count;
    const float* llr = mio->llr;
    const int64_t* off = mio->off;
    const int64_t stride = num_groups_x() * G::FPW;
    for (int64_t q0 = gid_x() * G::FPW; q0 < cnt; q0 += stride) {
        const int64_t q = q0 + slot;
        if (G::T >= 64) __syncthreads();  // the previous frame's staging is read
        if (q >= cnt) break;             // only when T < 64: this slot's wavefront lanes leave alone
        const int id = ids[q];
        const CodeDev cd = mio->codes ? mio->codes[mio->code_of[id]] : code;
        FrameIO io;
        io.llr = llr + off[id];
        io.u_hat = u_hat + (int64_t)id * u_stride;
        io.info = nullptr;
        io.llr_u = nullptr;
        io.iters = iters_out + id;
        io.ok = ok_out + id;
        io.saved = nullptr;
        const bool okv = bp_frame<G, WEIGHTED, false>(cd, io, max_iter, stop, lmax, W, sh, t, slot);
        if (t == 0 && !okv) fail_ids[atomicAdd(fail_count, 1)] = id;
    }
}

// ------------------------------------------------------------------ dispatch

using KernelFn = void (*)(CodeDev, const float*, int64_t, int, int, float, const float*, uint8_t*, uint8_t*,
                          float*, int32_t*, uint8_t*, float*);

using GatherFn = void (*)(CodeDev, const MixedIo*, const int32_t*, const int32_t*, int, int, float, const float*,
                          uint8_t*, int64_t, int32_t*, uint8_t*, int32_t*, int32_t*);

struct Entry {
    KernelFn plain, weighted, weighted_save, exact, weighted_stage;
    KernelFn persist_plain, persist_weighted_stage;
    GatherFn gather_plain, gather_weighted;
    int wg, fpw;
};

template <int NL, int RL>
constexpr Entry make_entry() {
    return Entry{&bp_kernel<NL, RL, false, false>, &bp_kernel<NL, RL, true, false>, &bp_kernel<NL, RL, true, true>,
                 &bp_kernel<NL, RL, false, false, 1>, &bp_kernel<NL, RL, true, false, 0, true>,
                 &bp_kernel<NL, RL, false, false, 0, false, true>, &bp_kernel<NL, RL, true, false, 0, true, true>,
                 &bp_gather_kernel<NL, RL, false>, &bp_gather_kernel<NL, RL, true>, Geom<NL, RL>::WG,
                 Geom<NL, RL>::FPW};
}

// variants: register bits r = 2 or 3 (variant id = r)
constexpr int kMinN = 3, kMaxN = 12;

const Entry* lookup(int n, int r) {
    static const Entry table[kMaxN + 1][4] = {
        {},
        {},
        {},
        {{}, {}, make_entry<3, 2>(), make_entry<3, 3>()},
        {{}, {}, make_entry<4, 2>(), make_entry<4, 3>()},
        {{}, {}, make_entry<5, 2>(), make_entry<5, 3>()},
        {{}, {}, make_entry<6, 2>(), make_entry<6, 3>()},
        {{}, {}, make_entry<7, 2>(), make_entry<7, 3>()},
        {{}, {}, make_entry<8, 2>(), make_entry<8, 3>()},
        {{}, {}, make_entry<9, 2>(), make_entry<9, 3>()},
        {{}, {}, make_entry<10, 2>(), make_entry<10, 3>()},
        {{}, {}, make_entry<11, 2>(), make_entry<11, 3>()},
        {{}, {}, make_entry<12, 2>(), make_entry<12, 3>()},
    };
    if (n < kMinN || n > kMaxN || r < 2 || r > 3) return nullptr;
    return &table[n][r];
}

}  // namespace bp

bool bp_variant_supported(int n, int variant) { return bp::lookup(n, variant) != nullptr; }

int bp_default_variant(int n) { return n >= 9 ? 3 : 2; }

int bp_list_variants(int n, int32_t* ids, int cap) {
    int c = 0;
    for (int r = 2; r <= 3; ++r)
        if (bp::lookup(n, r)) {
            if (ids && c < cap) ids[c] = r;
            ++c;
        }
    return c;
}

polar_status launch_bp(const polar_code* code, const float* llr, int64_t B, const bp_params* p, uint8_t* u_hat,
                       float* llr_u, int32_t* iters, uint8_t* ok, hipStream_t stream, int wgs_per_cu,
                       uint8_t* info_out) {
    const int variant = p->variant ? p->variant : bp_default_variant(code->n);
    const bp::Entry* e = bp::lookup(code->n, variant);
    if (!e) return set_error(POLAR_ERR_UNSUPPORTED, "bp: no kernel variant for this block length");
    if (B == 0) return POLAR_OK;
    const int64_t blocks = (B + e->fpw - 1) / e->fpw;
    if (blocks > (int64_t)INT32_MAX) return set_error(POLAR_ERR_INVALID_ARG, "bp: batch too large");
    bp::KernelFn fn = p->rule == 1 ? e->exact
                      : !p->weights        ? e->plain
                      : p->weight_layout   ? e->weighted_stage
                                           : e->weighted;
    int64_t grid = blocks;
    if (wgs_per_cu > 0 && p->rule == 0 && (!p->weights || p->weight_layout == 1)) {
        // capped persistent grid: leaves room on every CU for concurrent kernels
        const int64_t cap = (int64_t)device_cu_count() * wgs_per_cu;
        if (cap < blocks) {
            fn = p->weights ? e->persist_weighted_stage : e->persist_plain;
            grid = cap;
        }
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(e->wg), 0, stream, code->dev(), llr, B, p->max_iter, p->stop,
                       p->llr_max, p->weights, u_hat, info_out, llr_u, iters, ok, (float*)nullptr);
    return hip_check(hipGetLastError(), "bp_kernel launch");
}

polar_status bp_gather_grid(const polar_code* code, const bp_params* p, int64_t max_frames, int* grid) {
    const int variant = p->variant ? p->variant : bp_default_variant(code->n);
    const bp::Entry* e = bp::lookup(code->n, variant);
    if (!e) return set_error(POLAR_ERR_UNSUPPORTED, "bp: no kernel variant for this block length");
    bp::GatherFn fn = p->weights ? e->gather_weighted : e->gather_plain;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, e->wg, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)device_cu_count() * per_cu;
    const int64_t need = (max_frames + e->fpw - 1) / e->fpw;
    if (need < g) g = need;
    *grid = (int)(g < 1 ? 1 : g);
    return POLAR_OK;
}

polar_status launch_bp_gather(const polar_code* code, const MixedIo* io, const int32_t* ids, const int32_t* count,
                              const bp_params* p, uint8_t* u_hat, int64_t u_stride, int32_t* iters, uint8_t* ok,
                              int32_t* fail_ids, int32_t* fail_count, int grid, hipStream_t stream) {
    const int variant = p->variant ? p->variant : bp_default_variant(code->n);
    const bp::Entry* e = bp::lookup(code->n, variant);
    if (!e) return set_error(POLAR_ERR_UNSUPPORTED, "bp: no kernel variant for this block length");
    bp::GatherFn fn = p->weights ? e->gather_weighted : e->gather_plain;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(e->wg), 0, stream, code->dev(), io, ids, count, p->max_iter,
                       p->stop, p->llr_max, p->weights, u_hat, u_stride, iters, ok, fail_ids, fail_count);
    return hip_check(hipGetLastError(), "bp_gather_kernel launch");
}

polar_status launch_bp_save(const polar_code* code, const float* llr, int64_t B, int T, float llr_max,
                            const float* W, int variant, uint8_t* u_hat, float* llr_u, uint8_t* ok, float* saved,
                            hipStream_t stream) {
    const int v = variant ? variant : bp_default_variant(code->n);
    const bp::Entry* e = bp::lookup(code->n, v);
    if (!e) return set_error(POLAR_ERR_UNSUPPORTED, "wbp: no kernel variant for this block length");
    if (B == 0) return POLAR_OK;
    const int64_t blocks = (B + e->fpw - 1) / e->fpw;
    bp::KernelFn fn = saved ? e->weighted_save : e->weighted;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(e->wg), 0, stream, code->dev(), llr, B, T, 0, llr_max, W,
                       u_hat, (uint8_t*)nullptr, llr_u, (int32_t*)nullptr, ok, saved);
    return hip_check(hipGetLastError(), "bp_kernel launch");
}

}  // namespace polarhip

using namespace polarhip;

extern "C" polar_status polar_bp_variants(int32_t N, int32_t* ids, int32_t cap, int32_t* count) {
    if (!count || cap < 0) return set_error(POLAR_ERR_INVALID_ARG, "polar_bp_variants: bad argument");
    int n = 0;
    while ((1 << n) < N) ++n;
    if ((1 << n) != N) return set_error(POLAR_ERR_INVALID_ARG, "polar_bp_variants: N not a power of two");
    *count = bp_list_variants(n, ids, cap);
    return ok_status();
}

extern "C" polar_status bp_decode_batch(const polar_code* code, const float* llr, int64_t B, const bp_params* p,
                                        uint8_t* u_hat, float* llr_u, int32_t* iters, uint8_t* ok,
                                        hipStream_t stream) {
    if (!code || !p) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: null code or params");
    if (B < 0) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: negative batch");
    if (B > 0 && (!llr || !u_hat || !ok)) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: null buffer");
    if (p->max_iter < 1) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: max_iter must be >= 1");
    if (p->stop < 0 || p->stop > 2) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: stop must be 0, 1 or 2");
    if (p->stop == 2 && code->c == 0)
        return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: CRC stop needs a code with a CRC");
    if (!(p->llr_max > 0.0f)) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: llr_max must be > 0");
    if (p->rule != 0 && p->rule != 1) return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: rule must be 0 or 1");
    if (p->rule == 1 && p->weights)
        return set_error(POLAR_ERR_UNSUPPORTED, "bp_decode_batch: the exact rule has no weighted form");
    if (p->weights && p->weight_iters < p->max_iter)
        return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: weight_iters < max_iter");
    if (p->weight_layout != 0 && p->weight_layout != 1)
        return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: weight_layout must be 0 or 1");
    if (p->variant != 0 && !bp_variant_supported(code->n, p->variant))
        return set_error(POLAR_ERR_INVALID_ARG, "bp_decode_batch: unknown variant");
    polar_status st = launch_bp(code, llr, B, p, u_hat, llr_u, iters, ok, stream);
    return st == POLAR_OK ? ok_status() : st;
}
