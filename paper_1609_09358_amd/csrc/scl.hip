// scl.hip -- CRC-aided successive-cancellation list decoder (Sec. II-A).
//
// One wavefront decodes one frame at a time; workgroups stay resident and walk
// a list of frames whose length may live on the device (the hybrid decoder
// feeds it the compacted BP failures without a host round trip).
//
// Path slot l is owned by lane l.  The LLR tree of a path (level d holds 2^d
// values, level n is the channel) and its partial sums (level d holds 2^d
// bits) are split in two:
//   - levels below BL = min(n, 5) live in the registers of the owning lane;
//   - level BL lives in LDS and the levels above it in the workgroup's global
//     slice (partial sums of levels >= 5 in LDS); they are shared lazily:
//     each slot keeps, per level, the slot whose array it reads.  Bit i rewrites levels ctz(i)..BL of every path into the
//     path's own slot and reads level ctz(i)+1 through the pointer, which no
//     path writes during bit i; partial sums are handled the same way.
// Bits are processed in blocks of 2^BL.  Inside a block, ctz(i) and the number
// of trailing ones of i are compile-time constants, so a block is unrolled
// into straight-line code: a bit recomputes levels ctz(i)..0 in registers
// (level BL is read from LDS at the block start and once in the middle),
// decides, and folds the decided bit into the partial sums held in registers.
// A branching path is copied by pulling from the parent's lane exactly the
// registers that later bits of the block still read, plus the two pointer
// vectors.  The candidates of a branching bit are listed parent by parent
// (bit 0 first); the L smallest under the strict order (metric, parent list
// position, bit) survive -- the pruned pseudo sort of Sec. II-A with a strict
// tie rule -- and keep that candidate order, so a survivor's slot is the
// number of survivors listed before it (found with a wavefront ballot) and
// slot index and list position coincide.  Which candidates survive is found
// by counting (each candidate counts the smaller ones), a bitonic sort across
// the wavefront, or threshold selection (the L-th smallest metric found bit by
// bit with ballots).  The CRC is tracked per path as a
// running syndrome (linear in the decided bits).  Each path carries its
// decided bits of the current block in a register word and the slot it held
// at the block start (both pulled from the parent on a branch); at every
// block end each path writes that pair to the trace, so the chosen path is
// recovered by one step per block (its slot at each block end), after which
// every lane writes its outputs from the block words.
//
// A frame's decode is a long chain of dependent steps, so throughput comes
// from many frames in flight: the kernel is held to 128 VGPRs (four waves per
// SIMD) and the LDS state is sized to let sixteen one-wave workgroups share a
// CU; the trace (5 bytes per block and path) moves to the workgroup's global
// slice when it does not fit.
#include <atomic>
#include <type_traits>

#include "internal.hpp"

namespace polarhip {
namespace scl {

// Min-sum f (the check-node rule with min-sum, Sec. II-A): sgn(a) sgn(b)
// min(|a|, |b|), as b clamped to [-|a|, |a|] with a's sign applied -- one med3
// and one bit operation; a zero result may carry the other sign, which no
// decision, penalty or metric depends on.
__device__ __forceinline__ float f_ms(float a, float b) {
    const float m = __builtin_amdgcn_fmed3f(b, -fabsf(a), fabsf(a));
    return __uint_as_float(__float_as_uint(m) ^ (__float_as_uint(a) & 0x80000000u));
}

// g(a, b) = b + (1 - 2u) a with the partial-sum bit u at bit position q of
// word w (q known at compile time where it is called): the bit moved onto
// a's sign, b - a being b + (-a), rounded alike
__device__ __forceinline__ float g_bit(float a, float b, uint32_t w, int q) {
    const uint32_t sb = (w << (31 - q)) & 0x80000000u;
    return b + __uint_as_float(__float_as_uint(a) ^ sb);
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

// Pointers typed by address space: LDS (3) and global (1).  Generic pointers
// would compile to flat instructions, whose waits also wait for every
// outstanding global access, and an LDS access through them takes the slower
// flat path; so LDS and global data are never reached through one pointer.
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;
template <typename T>
using glb_ptr = __attribute__((address_space(1))) T*;

// plain 4-lane vectors (the HIP vector classes do not bind to pointers of a
// named address space)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ lds_ptr<T> as_lds(void* p) {
    return (lds_ptr<T>)p;
}
template <typename T>
__device__ __forceinline__ glb_ptr<T> as_glb(const void* p) {
    return (glb_ptr<T>)const_cast<void*>(p);
}

// a value every lane holds alike, moved to scalar registers (so what is read
// through it becomes scalar or uniform-address work)
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ glb_ptr<T> uniform_glb(glb_ptr<T> p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (glb_ptr<T>)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// the slot read at each shared level, one byte per level: only levels 5..12
// are shared through slots (levels below 5 live in registers, N <= 4096), so
// eight bytes, one 64-bit register pair, hold them all (a branch pulls one
// pair per vector from the parent)
struct PtrVec {
    uint64_t w;
};

__device__ __forceinline__ int get_byte(const PtrVec& v, int idx) {
    const int sh = idx > 5 ? 8 * (idx - 5) : 0;  // levels below 5 are never read here
    return (int)((v.w >> sh) & 0xFFull);
}

__device__ __forceinline__ void set_byte(PtrVec& v, int idx, int val) {
    const int sh = idx > 5 ? 8 * (idx - 5) : 0;
    v.w = (v.w & ~(0xFFull << sh)) | ((uint64_t)val << sh);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    return (uint64_t)__shfl((unsigned long long)v, src, 64);
}

// word offset of partial-sum level d >= 5 inside a slot's LDS words
__device__ __forceinline__ int ps_off(int d) { return (1 << (d - 5)) - 1; }

constexpr int ctz_c(int v) {
    int c = 0;
    while (((v >> c) & 1) == 0) ++c;
    return c;
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// partial-sum block of 2^T bits finished by `bit`, from the T levels below it
template <int T>
__device__ __forceinline__ uint32_t combine(uint32_t bit, const uint32_t (&ps)[5]) {
    uint32_t cur = bit;
#pragma unroll
    for (int d = 0; d < T; ++d) {
        const uint32_t h = 1u << d;
        const uint32_t lowmask = (h >= 32u) ? 0xFFFFFFFFu : ((1u << h) - 1u);
        cur = ((ps[d] ^ cur) & lowmask) | (cur << h);
    }
    return cur;
}

// rank of this lane's candidate among the first ncand lanes under
// (metric, lane); metrics are non-negative, so their bit patterns order them.
// The metrics go through LDS once; each lane then reads them back as uint4
// broadcasts, four at a time, so the reads overlap.
template <int L>
__device__ __forceinline__ int candidate_rank(lds_ptr<uint32_t> mets, int ncand, float met, int lane) {
    constexpr int NC = 2 * L;
    constexpr int G = NC / 4 < 1 ? 1 : (NC / 4 > 4 ? 4 : NC / 4);  // uint4 reads in flight
    if (lane < ncand) mets[lane] = __float_as_uint(met);
    wave_mem_order();
    const uint32_t mb = __float_as_uint(met);
    int rank = 0;
    for (int c0 = 0; c0 < ncand; c0 += 4 * G) {
        u32x4 v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = ((lds_ptr<const u32x4>)(mets + c0))[g];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = c0 + 4 * g;
            rank += (c + 0 < ncand && (v[g].x < mb || (v[g].x == mb && c + 0 < lane))) ? 1 : 0;
            rank += (c + 1 < ncand && (v[g].y < mb || (v[g].y == mb && c + 1 < lane))) ? 1 : 0;
            rank += (c + 2 < ncand && (v[g].z < mb || (v[g].z == mb && c + 2 < lane))) ? 1 : 0;
            rank += (c + 3 < ncand && (v[g].w < mb || (v[g].w == mb && c + 3 < lane))) ? 1 : 0;
        }
    }
    return rank;
}

// Bitonic sorting network over the candidates across the wavefront (the
// alternative to the pruned pseudo sort that Sec. II-A also describes): keys
// (metric bits, lane) in the same strict order as candidate_rank, lanes
// without a candidate last; only the stages that separate the L smallest keys
// from the rest are run (survivors keep the candidate order, so the order
// among them is not needed).

// The keys of lane and of lane ^ J, all in VALU: data-parallel-primitive
// moves inside a row of 16 lanes for J <= 8 (J = 1, 2: one quad permute;
// J = 4: half-row mirror, then quad reversal; J = 8: row mirror, then
// half-row mirror), giving (own, partner); for J = 16, 32 the gfx950 row
// swaps, which exchange the upper rows of their first operand with the lower
// rows of the second -- with the key in both, every lane ends up holding its
// own key and its partner's, in an order that depends on the lane, which a
// compare-exchange does not need to know.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    if constexpr (J == 1) {
        return dpp_mov<0xB1>(v);  // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]
    } else if constexpr (J == 4) {
        return dpp_mov<0x1B>(dpp_mov<0x141>(v));  // half mirror, quad_perm [3,2,1,0]
    } else {
        static_assert(J == 8, "distance");
        return dpp_mov<0x141>(dpp_mov<0x140>(v));  // row mirror, half mirror
    }
}

template <int J>
__device__ __forceinline__ void key_pair(uint32_t lo, uint32_t hi, uint64_t& a, uint64_t& b) {
    if constexpr (J <= 8) {
        a = ((uint64_t)hi << 32) | lo;
        b = ((uint64_t)lane_xor<J>(hi) << 32) | lane_xor<J>(lo);
    } else if constexpr (J == 16) {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a = ((uint64_t)rh[0] << 32) | rl[0];
        b = ((uint64_t)rh[1] << 32) | rl[1];
    } else {
        static_assert(J == 32, "distance");
        const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a = ((uint64_t)rh[0] << 32) | rl[0];
        b = ((uint64_t)rh[1] << 32) | rl[1];
    }
}

// one compare-exchange at distance J while merging runs into sorted runs of
// K: the lane keeps the smaller key of {a, b} or the larger, by its position
// (keys are distinct: every one carries its lane)
template <int K, int J>
__device__ __forceinline__ void bitonic_cx(uint32_t& lo, uint32_t& hi, int lane) {
    uint64_t a, b;
    key_pair<J>(lo, hi, a, b);
    const bool keep_max = ((lane & K) == 0) != ((lane & J) == 0);
    const uint64_t r = ((b < a) != keep_max) ? b : a;
    lo = (uint32_t)r;
    hi = (uint32_t)(r >> 32);
}

// the stages J = K/2 .. 1 that merge bitonic runs into sorted runs of K
template <int K, int J>
__device__ __forceinline__ void bitonic_merge(uint32_t& lo, uint32_t& hi, int lane) {
    bitonic_cx<K, J>(lo, hi, lane);
    if constexpr (J > 1) bitonic_merge<K, J / 2>(lo, hi, lane);
}

// every merge from runs of 2 up to sorted runs of K_END, in alternating
// directions
template <int K, int K_END>
__device__ __forceinline__ void bitonic_merge_upto(uint32_t& lo, uint32_t& hi, int lane) {
    bitonic_merge<K, K / 2>(lo, hi, lane);
    if constexpr (K < K_END) bitonic_merge_upto<K * 2, K_END>(lo, hi, lane);
}

// The L smallest keys of lanes 0..2L-1 gathered in lanes 0..L-1, in no
// particular order (lanes without a candidate carry the largest keys): the
// bitonic sort's merges up to sorted runs of L, which leave lanes 0..2L-1 one
// bitonic sequence, then the first compare-exchange of the next merge, at
// distance L, which puts the smaller key of each pair below -- the sort's
// remaining stages would only order the halves.  Returns the lane of the
// candidate whose key this lane now holds (the keys stay a permutation of the
// lanes' own).
template <int L>
__device__ __forceinline__ int bitonic_partition(float met, int ncand, int lane) {
    uint32_t hi = lane < ncand ? __float_as_uint(met) : 0xFFFFFFFFu;
    uint32_t lo = (uint32_t)lane;
    bitonic_merge_upto<2, L>(lo, hi, lane);
    bitonic_cx<2 * L, L>(lo, hi, lane);
    return (int)(lo & 63u);
}

// set bits of a wavefront mask, counted in two 32-bit halves (a uniform
// 32-bit count keeps the comparisons that use it in scalar instructions)
__device__ __forceinline__ uint32_t mask_count(uint64_t m) {
    return (uint32_t)__builtin_popcount((uint32_t)m) + (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
}

// set bits of a wavefront mask below this lane
__device__ __forceinline__ int mask_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Threshold selection: whether this lane's candidate is among the L smallest
// of the ncand > L candidates under (metric, lane).  The L-th smallest metric
// tau is found bit by bit from the top (metrics are non-negative, so their
// bit patterns order them): the largest value with fewer than L metrics
// below it.  Candidates below tau survive, and of those equal to tau the
// lowest lanes, as many as are still missing.  One compare per bit in VALU;
// the counts are scalar.
template <int L>
__device__ __forceinline__ bool threshold_keep(float met, int ncand, int lane) {
    const uint32_t key = lane < ncand ? __float_as_uint(met) : 0xFFFFFFFFu;
    uint32_t tau = 0u;
#pragma unroll
    for (int b = 30; b >= 0; --b) {
        const uint32_t trial = tau | (1u << b);
        tau = mask_count(__ballot(key < trial)) < (uint32_t)L ? trial : tau;
    }
    const int need = L - (int)mask_count(__ballot(key < tau));
    const uint64_t eq = __ballot(key == tau);
    return key < tau || (key == tau && mask_below(eq) < need);
}

// ranking of the candidates: the pruned pseudo sort (each candidate counts
// those before it), a bitonic sort, or threshold selection
enum : int { kRankCount = 0, kRankBitonic = 1, kRankThreshold = 2 };

// The survivors of one branching bit.  Lane c holds candidate c (parent
// c >> 1 of the list, bit c & 1) with metric met, c < ncand.  Which
// candidates survive follows the strict order (metric, parent, bit); the
// survivors keep the candidate order, so the new list's slot s holds the s-th
// surviving candidate.  Returns, for lane s, the lane of that candidate
// (lanes past the new list size get a discarded candidate, whose state no one
// reads).
template <int L, int RANK>
__device__ __forceinline__ int select_survivors(lds_ptr<uint32_t> mets, float met, int ncand, int lane) {
    if (ncand <= L) return lane;  // every candidate survives in place
    bool keep;
    if constexpr (RANK == kRankCount) {
        keep = lane < ncand && candidate_rank<L>(mets, ncand, met, lane) < L;
    } else if constexpr (RANK == kRankBitonic) {
        // lanes 0..L-1 hold the L smallest candidates and tell them so
        const int c = bitonic_partition<L>(met, ncand, lane);
        keep = __builtin_amdgcn_ds_permute(c << 2, lane < L ? 1 : 0) != 0;
    } else {
        keep = threshold_keep<L>(met, ncand, lane);
    }
    // exactly L survivors: they go to slots 0..L-1 in lane order, the others
    // to L..63, so the push below has distinct destinations
    const uint64_t m = __ballot(keep);
    const int dest = keep ? mask_below(m) : L + mask_below(~m);
    return __builtin_amdgcn_ds_permute(dest << 2, lane);
}

struct Layout {
    int gl;      // LLR levels < gl in LDS (gl = min(n, 6)), the others in the workgroup's global slice
    int sl;      // LDS floats per slot: levels BL..gl-1, level d at offset 2^d - 2^BL, padded
    int pw;      // partial-sum words per slot (levels >= 5)
    int tg;      // 1: the trace lives in the global slice and is read back in chunks
    int64_t gbytes;  // bytes of the global slice per workgroup
    int64_t toff;    // byte offset of the trace inside the slice
    int tboff;       // byte offset of the LDS trace (the traceback's block chain sits below it)
    int nblk;        // blocks of the largest block length the layout holds (trace rows)
    int64_t u_stride;  // u_hat row stride of a ragged batch
};

// Levels top..5 of every path at a block start (top = the highest level whose
// index bit changed).  Level 5 of a path is 32 items, taken as eight groups of
// four; group g of path p is one chain, run by lane 8 (p mod 8) + g as its
// chain p / 8.  A chain's items of level d are the items e + 32 k of its group
// e, and each depends only on the same chain's items of level d + 1, so a
// lane computes its chains from level top + 1 alone, in registers: the level
// top items are the leaves, taken in bit-reversed order so that each pair of
// consecutive results at one level combines at once into the level below
// (a stack of one pending value per level); every item is stored on the way
// for the later bits and blocks (level 5 in LDS, the levels above in the
// workgroup's global slice), and nothing stored here is read back here.
// The chains of a lane run as one stream of leaves, the loads of the next P
// leaves in flight (two where the stack is deep, N >= 2048, to stay within the
// register budget).  Every load is issued unconditionally (a load past the
// stream's end repeats the last leaf's), so the waits for one leaf's data
// leave the later leaves' loads outstanding.  With L >= 8 the chains of
// paths past the list's end (slots below 8 * chains <= L) store too: those
// slots' levels top..5 are rewritten before any path reads them.  H = top - 5.
struct Leaf {
    f32x4 a, b;   // items e and e + 2^top of level top + 1
    uint32_t w;   // partial-sum bits of the four items (g at the top level)
};

template <int L, int H, bool CHAN1>
__device__ __forceinline__ void block_levels(const int act, const int lane, const int N, const int SL, const int PW,
                                             const lds_ptr<float> slam, const glb_ptr<float> glam,
                                             const glb_ptr<const float> gsrc, const int gstride,
                                             const lds_ptr<uint32_t> psw, const bool psum, const uint32_t srcpack,
                                             const uint32_t psspack) {
    constexpr int TOP = H + 5;
    constexpr int M = 1 << H;             // leaves per chain
    constexpr int P = H <= 4 ? 4 : 2;     // leaves in flight
    constexpr int LP = P == 4 ? 2 : 1;    // log2 P
    constexpr int SZT = 1 << TOP;
    const int C = (act + 7) >> 3;         // chains per lane
    const int S = C << H;                 // leaves per lane
    // the lane index made opaque here, so that the lane offsets below are
    // computed at each block start instead of being hoisted out of the frame
    // loop and held in registers throughout
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int e4 = (ln & 7) << 2;         // the group's first item
    auto leaf_k = [](int m) -> int { return H == 0 ? 0 : (int)(__builtin_bitreverse32((uint32_t)m) >> (32 - H)); };
    auto load = [&](int st) -> Leaf {
        Leaf o;
        const int c = st >> H;
        const int k = leaf_k(st & (M - 1));
        const int it = e4 + 32 * k;
        if constexpr (!CHAN1) {
            // level top + 1 of the chain's source slot (stride 0: the channel
            // row), 32-bit byte offsets from the uniform base
            const int src = (int)((srcpack >> (8 * c)) & 0xFFu);
            const uint32_t off = (uint32_t)(src * gstride + it) * 4u;
            o.a = *(glb_ptr<const f32x4>)((glb_ptr<const char>)gsrc + off);
            o.b = *(glb_ptr<const f32x4>)((glb_ptr<const char>)gsrc + off + 4u * SZT);
        } else {
            const glb_ptr<const float> q = gsrc + it;
            o.a = f32x4{q[0], q[1], q[2], q[3]};
            o.b = f32x4{q[SZT], q[SZT + 1], q[SZT + 2], q[SZT + 3]};
        }
        // the partial sums (read also where they are not used: the slot
        // pointers of the first block are valid)
        const int pss = (int)((psspack >> (8 * c)) & 0xFFu);
        o.w = psw[pss * PW + ps_off(TOP) + k] >> e4;
        return o;
    };
    Leaf ring[P];
    f32x4 stk[H > 0 ? H : 1];
    // leaf s0 + q, s0 a multiple of P: the chain and the low bits of the leaf's
    // index in it are known at compile time where the chain is at least P long
    auto step = [&](const int s0, auto QC, Leaf& slotq) {
        constexpr int q = decltype(QC)::value;
        const Leaf x = slotq;
        slotq = load(s0 + q + P < S ? s0 + q + P : S - 1);
        const int m = M >= P ? ((s0 & (M - 1)) | q) : (q & (M - 1));
        const int c = M >= P ? (s0 >> H) : ((s0 >> H) + (q >> H));
        const int k = leaf_k(m);
        const int slot = (ln >> 3) + 8 * c;
        const bool live = L >= 8 || slot < act;
        auto put = [&](auto DC, int kk, const f32x4& v) {
            constexpr int d = decltype(DC)::value;
            if (!live) return;
            if constexpr (d == 5) *(lds_ptr<f32x4>)(slam + slot * SL + e4 + 32 * kk) = v;
            else *(glb_ptr<f32x4>)((glb_ptr<char>)glam + (uint32_t)(slot * N + (1 << d) + e4 + 32 * kk) * 4u) = v;
        };
        f32x4 v;
        if (psum) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = g_bit(x.a[i], x.b[i], x.w, i);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = f_ms(x.a[i], x.b[i]);
        }
        put(std::integral_constant<int, TOP>{}, k, v);
        bool go = true;
        static_for<0, H>([&](auto LC) {
            constexpr int l = decltype(LC)::value;
            // bit l of the leaf's index: compile-time below log2 P
            const bool one = (M >= P && l < LP) ? ((q >> l) & 1) != 0 : ((m >> l) & 1) != 0;
            if (go) {
                if (one) {
                    f32x4 u;
#pragma unroll
                    for (int i = 0; i < 4; ++i) u[i] = f_ms(stk[l][i], v[i]);
                    v = u;
                    put(std::integral_constant<int, TOP - l - 1>{}, k & ((M >> (l + 1)) - 1), v);
                } else {
                    stk[l] = v;
                    go = false;
                }
            }
        });
    };
#pragma unroll
    for (int q = 0; q < P; ++q) ring[q] = load(q < S ? q : S - 1);
    if (S % P == 0) {
        for (int s0 = 0; s0 < S; s0 += P)
            static_for<0, P>([&](auto QC) { step(s0, QC, ring[decltype(QC)::value]); });
    } else {
        // a stream not a multiple of P (fewer than 25 paths, lowest levels)
        for (int s0 = 0; s0 < S; s0 += P)
            static_for<0, P>([&](auto QC) {
                if (s0 + decltype(QC)::value < S) step(s0, QC, ring[decltype(QC)::value]);
            });
    }
}

template <int L, int BL, int RANK = kRankCount>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void scl_kernel(CodeDev code_in, const float* __restrict__ llr,
                                                 const int32_t* __restrict__ frame_ids,
                                                 const int32_t* __restrict__ count_dev, int64_t count_host,
                                                 uint8_t* __restrict__ u_hat, uint8_t* __restrict__ crc_ok,
                                                 float* __restrict__ pm_out, unsigned char* __restrict__ glob_all,
                                                 Layout lay, const MixedIo* __restrict__ mio) {
    constexpr int BS = 1 << BL;  // bits per block
    extern __shared__ __attribute__((aligned(16))) unsigned char sm[];
    const int lane = lid_x();
    const int gl = lay.gl, SL = lay.sl, PW = lay.pw;

    const lds_ptr<float> slam = as_lds<float>(sm);                          // [L][SL]
    const lds_ptr<uint32_t> psw = (lds_ptr<uint32_t>)(slam + L * SL);       // [L][PW]
    const lds_ptr<uint32_t> mets = psw + L * PW;                            // [64]
    const lds_ptr<int> chain = as_lds<int>(sm);                             // [nblk], reuses the LLR area at the end

    unsigned char* gbase = glob_all ? glob_all + (size_t)gid_x() * (size_t)lay.gbytes : nullptr;
    const glb_ptr<float> glam = as_glb<float>(gbase);         // [L][N], levels >= gl
    // the trace, per block and slot: the block's decided bits (bit r = bit r of
    // the block) and the slot the path held at the block start; in LDS or, when
    // tg, in the global slice
    const size_t tra_off = (size_t)lay.nblk * L * sizeof(uint32_t);
    const lds_ptr<uint32_t> tru_l = as_lds<uint32_t>(sm + lay.tboff);   // [nblk][L]
    const lds_ptr<uint8_t> tra_l = as_lds<uint8_t>(sm + lay.tboff + tra_off);
    const glb_ptr<uint32_t> tru_g = as_glb<uint32_t>(gbase + lay.toff);
    const glb_ptr<uint8_t> tra_g = as_glb<uint8_t>(gbase + lay.toff + tra_off);
    const bool tg = lay.tg != 0;

    const int64_t count = count_dev ? (int64_t)(*count_dev) : count_host;
    const float* const llr_base = mio ? mio->llr : llr;
    const int64_t* const row_off = mio ? mio->off : nullptr;
    for (int64_t q = gid_x(); q < count; q += num_groups_x()) {
        const int64_t f = frame_ids ? (int64_t)uniform_int(frame_ids[q]) : q;
        // the frame's code (several codes in one launch: the layout holds the
        // largest; level offsets inside a slot do not depend on n)
        CodeDev code = code_in;
        if (mio && mio->codes) {
            code = mio->codes[uniform_int(mio->code_of[f])];
            code.frozen_bits = uniform_ptr(code.frozen_bits);
            code.da_bits = uniform_ptr(code.da_bits);
            code.syn = uniform_ptr(code.syn);
            code.n = uniform_int(code.n);
            code.N = uniform_int(code.N);
        }
        const int n = code.n, N = code.N;
        // the frame's frozen and decision-aided words, lane w holding word w
        // (and word 64 + w): a block reads its word from the lanes
        const int nw = N >= 32 ? N >> 5 : 1;
        const glb_ptr<const uint32_t> fzb = as_glb<const uint32_t>(code.frozen_bits);
        const glb_ptr<const uint32_t> dab = as_glb<const uint32_t>(code.da_bits);
        const uint32_t fzv0 = lane < nw ? fzb[lane] : 0u, fzv1 = 64 + lane < nw ? fzb[64 + lane] : 0u;
        const uint32_t dav0 = lane < nw ? dab[lane] : 0u, dav1 = 64 + lane < nw ? dab[64 + lane] : 0u;
        const glb_ptr<const uint32_t> synp = as_glb<const uint32_t>(code.syn);
        // rows of frame f: LLRs at row_off[f] (ragged batch) or f * N; u_hat at
        // f * u_stride (ragged batch) or f * N
        const float* const chan_g = llr_base + (row_off ? row_off[f] : f * N);
        const glb_ptr<const float> chan = as_glb<const float>(chan_g);
        const bool chan16 = (reinterpret_cast<uintptr_t>(chan_g) & 15u) == 0;  // 16-byte loads possible
        const int64_t urow = f * (row_off ? lay.u_stride : (int64_t)N);

        int act = 1;
        float PM = 0.0f;
        uint32_t SYN = 0u;
        PtrVec ptrL{0ull};  // slot read at each LLR level >= BL
        PtrVec ptrP{0ull};  // slot read at each partial-sum level >= 5
        float lv[32];             // levels 0..BL-1, heap order: level d at [2^d, 2^(d+1))
        uint32_t ps[5];           // partial-sum levels 0..BL-1: bit e of word d
#pragma unroll
        for (int e = 0; e < 32; ++e) lv[e] = 0.0f;
#pragma unroll
        for (int d = 0; d < 5; ++d) ps[d] = 0u;
        uint32_t ublk = 0u;  // this path's decided bits of the current block
        int anc = lane;      // the slot this path held at the block start

        for (int j = 0; j < (N >> BL); ++j) {
            const int i0 = j << BL;
            const uint32_t bmask = BS == 32 ? 0xFFFFFFFFu : ((1u << BS) - 1u);
            const int wi = i0 >> 5;
            const uint32_t fword = (uint32_t)__builtin_amdgcn_readlane((int)(wi < 64 ? fzv0 : fzv1), wi & 63);
            const uint32_t dword = (uint32_t)__builtin_amdgcn_readlane((int)(wi < 64 ? dav0 : dav1), wi & 63);
            const uint32_t fw = (fword >> (i0 & 31)) & bmask;
            const uint32_t dw = (dword >> (i0 & 31)) & bmask;  // decision-aided
            // the block's CRC syndromes, lane r holding position i0 + r (loaded
            // after the block start's fence, which would otherwise wait for it)
            uint32_t synv = 0u;
            bool syn_loaded = false;
            // ---------------- block start: levels top..BL of every path
            if constexpr (BL == 5) {
                if (BL < n) {
                    const int top = (j == 0) ? n - 1 : __builtin_ctz((unsigned)i0);
                    // slots read at level top + 1 and partial sums at level top,
                    // of each chain's path: byte c for chain c of this lane
                    const int myp = get_byte(ptrL, top + 1);
                    const int mypp = get_byte(ptrP, top);
                    uint32_t srcpack = 0u, psspack = 0u;
#pragma unroll
                    for (int c = 0; c < (L + 7) / 8; ++c) {
                        const int pth = (lane >> 3) + 8 * c;
                        srcpack |= (uint32_t)__shfl(myp, pth, 64) << (8 * c);
                        psspack |= (uint32_t)__shfl(mypp, pth, 64) << (8 * c);
                    }
                    const bool psum = j != 0;
                    // level top + 1: the channel row (same for every path) or
                    // the workgroup's global slice
                    const bool in_chan = top + 1 == n;
                    const bool chan1 = in_chan && !chan16;
                    const glb_ptr<const float> gsrc =
                        uniform_glb(in_chan ? chan : (glb_ptr<const float>)(glam + (2 << top)));
                    const int gstride = in_chan ? 0 : N;
                    // the levels above were written by other lanes at earlier
                    // block starts
                    wg_mem_order();
                    synv = synp[i0 + (lane & (BS - 1))];
                    syn_loaded = true;
#define POLAR_BLOCK_LEVELS(HH)                                                                                   \
    (chan1 ? block_levels<L, HH, true>(act, lane, N, SL, PW, slam, glam, gsrc, gstride, psw, psum, srcpack, psspack) \
           : block_levels<L, HH, false>(act, lane, N, SL, PW, slam, glam, gsrc, gstride, psw, psum, srcpack, psspack))
                    switch (top - BL) {
                        case 0: POLAR_BLOCK_LEVELS(0); break;
                        case 1: POLAR_BLOCK_LEVELS(1); break;
                        case 2: POLAR_BLOCK_LEVELS(2); break;
                        case 3: POLAR_BLOCK_LEVELS(3); break;
                        case 4: POLAR_BLOCK_LEVELS(4); break;
                        case 5: POLAR_BLOCK_LEVELS(5); break;
                        default: POLAR_BLOCK_LEVELS(6); break;
                    }
#undef POLAR_BLOCK_LEVELS
                    // level 5 (LDS) is read by the block's bits
                    wave_mem_order();
                    if (lane < act)
                        for (int d = top; d >= BL; --d) set_byte(ptrL, d, lane);
                }
            }
            if (!syn_loaded) synv = synp[i0 + (lane & (BS - 1))];
            // the block's register levels and partial sums are all rewritten
            // before they are read again (lanes that join the list during the
            // block pull what they read): they carry nothing from the last block,
            // and the block start above had their registers
#pragma unroll
            for (int e = 0; e < 32; ++e) lv[e] = 0.0f;
#pragma unroll
            for (int d = 0; d < 5; ++d) ps[d] = 0u;
            ublk = 0u;
            anc = lane;
            // ---------------- the 2^BL bits of the block, unrolled
            static_for<0, BS>([&](auto RC) {
                constexpr int r = decltype(RC)::value;
                // lowest level whose index bit changed at this bit (BL: block start)
                constexpr int top = (r == 0) ? BL : ctz_c(r);
                // register level d (1 <= d < BL) is read next by the bit
                // r' = r - (r mod 2^d) + 2^(d-1) and rewritten by bit
                // r - (r mod 2^d) + 2^d: after bit r it is still to be read
                // exactly when bit d - 1 of r is clear
                constexpr unsigned live_levels = (r + 1 < BS) ? (~(unsigned)r & ((1u << (BL - 1)) - 1u)) : 0u;
                // trailing ones of the bit index (>= BL at the block's last bit)
                constexpr int tb = (r + 1 < BS) ? ctz_c(~r) : BL;

                // ---- LLR levels min(top, BL-1)..0 of this lane's path
                if (lane < act) {
                    float src[32];
                    constexpr int sl_lv = (r == 0) ? BL : top + 1;  // level read
                    if constexpr (sl_lv == BL) {
                        if (BL == n) {
#pragma unroll
                            for (int e = 0; e < BS; ++e) src[e] = chan[e];
                        } else {
                            const int sl = (r == 0) ? lane : get_byte(ptrL, BL);
                            const lds_ptr<float> p = slam + sl * SL;
#pragma unroll
                            for (int e4 = 0; e4 < BS / 4; ++e4) {
                                const f32x4 t4 = ((lds_ptr<const f32x4>)p)[e4];
                                src[4 * e4] = t4.x;
                                src[4 * e4 + 1] = t4.y;
                                src[4 * e4 + 2] = t4.z;
                                src[4 * e4 + 3] = t4.w;
                            }
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < (1 << sl_lv); ++e) src[e] = lv[(1 << sl_lv) + e];
                    }
                    constexpr int dhi = sl_lv - 1;  // first level computed here
#pragma unroll
                    for (int d = dhi; d >= 0; --d) {
#pragma unroll
                        for (int e = 0; e < (1 << d); ++e) {
                            const float a = (d == dhi) ? src[e] : lv[(2 << d) + e];
                            const float b = (d == dhi) ? src[e + (1 << d)] : lv[(2 << d) + e + (1 << d)];
                            if (r != 0 && d == top)
                                lv[(1 << d) + e] = g_bit(a, b, ps[d], e);
                            else
                                lv[(1 << d) + e] = f_ms(a, b);
                        }
                    }
                }
                const float lam0 = lv[1];
                // ---- decision
                uint32_t bit = 0;
                if ((fw >> r) & 1u) {
                    if (lane < act) PM = PM + (lam0 < 0.0f ? fabsf(lam0) : 0.0f);
                } else if ((dw >> r) & 1u) {
                    // decision-aided position (Sec. II-A): every path keeps its
                    // hard decision; no branching, no metric change, same slots
                    if (lane < act) {
                        bit = lam0 < 0.0f ? 1u : 0u;
                        SYN ^= bit ? (uint32_t)__builtin_amdgcn_readlane((int)synv, r) : 0u;
                        ublk |= bit << r;
                    }
                } else {
                    const int ncand = 2 * act;
                    const int p = lane >> 1, b = lane & 1;
                    const float lp = __shfl(lam0, p, 64);
                    const float pmp = __shfl(PM, p, 64);
                    const float pen = (b != (lp < 0.0f ? 1 : 0)) ? fabsf(lp) : 0.0f;
                    const float met = pmp + pen;
                    const int nact = ncand < L ? ncand : L;
                    const int c = select_survivors<L, RANK>(mets, met, ncand, lane);
                    const int par = c >> 1;
                    const uint32_t cb = (uint32_t)(c & 1);
                    const uint32_t syn_i = (uint32_t)__builtin_amdgcn_readlane((int)synv, r);
                    // pull the parent's state: metric, syndrome, pointers, live registers
                    // (lanes past the new list size pull lane 0's state, which no one reads)
                    PM = __shfl(met, c, 64);
                    SYN = __shfl(SYN, par, 64) ^ (cb ? syn_i : 0u);
                    ptrL.w = shfl64(ptrL.w, par);
                    ptrP.w = shfl64(ptrP.w, par);
                    // partial-sum level d is written at the bits r with r mod
                    // 2^(d+1) = 2^d - 1 and read at those with r mod 2^(d+1) in
                    // [2^d, 2^(d+1) - 1] (g at level d, then the fold at the
                    // end of the 2^(d+1) block): after this point it is still to
                    // be read exactly when bit d of r is set
                    static_for<0, BL>([&](auto DC) {
                        constexpr int d = decltype(DC)::value;
                        if constexpr ((r >> d) & 1) ps[d] = __shfl(ps[d], par, 64);
                    });
                    static_for<1, BL>([&](auto DC) {
                        constexpr int d = decltype(DC)::value;
                        if constexpr ((live_levels >> (d - 1)) & 1u) {
#pragma unroll
                            for (int e = 1 << d; e < (2 << d); ++e) lv[e] = __shfl(lv[e], par, 64);
                        }
                    });
                    anc = __shfl(anc, par, 64);
                    ublk = __shfl(ublk, par, 64) | (cb << r);
                    if (lane < nact) bit = cb;
                    act = nact;
                }
                // ---- partial sums: the finished block of 2^t bits becomes level t
                if constexpr (tb < BL) {
                    if (lane < act) ps[tb] = combine<tb>(bit, ps);
                } else {
                    const int t = (BL == n) ? n : BL + __builtin_ctz(~(unsigned)j);
                    if (t < n) {
                        // level t >= 5 lives in LDS: W = 2^(t-5) words built in place
                        // from the end, starting with this 32-bit block
                        const int W = 1 << (t - 5);
                        const int ot = ps_off(t);
                        if (lane < act) psw[lane * PW + ot + W - 1] = combine<BL>(bit, ps);
                        wave_mem_order();
                        for (int d = 5; d < t; ++d) {
                            const int sz = 1 << (d - 5);
                            const int items = act * sz;
                            const int mypp = get_byte(ptrP, d);
                            for (int it = lane; it < items; it += 64) {
                                const int slot = it >> (d - 5), w = it & (sz - 1);
                                const int pss = __shfl(mypp, slot, 64);
                                const uint32_t v = psw[pss * PW + ps_off(d) + w] ^ psw[slot * PW + ot + W - sz + w];
                                psw[slot * PW + ot + W - 2 * sz + w] = v;
                            }
                            wave_mem_order();
                        }
                        if (lane < act) set_byte(ptrP, t, lane);
                        wave_mem_order();
                    }
                }
            });
            // ---- the block's trace entry of every path
            if (lane < act) {
                if (tg) {
                    tru_g[j * L + lane] = ublk;
                    tra_g[j * L + lane] = (uint8_t)anc;
                } else {
                    tru_l[j * L + lane] = ublk;
                    tra_l[j * L + lane] = (uint8_t)anc;
                }
            }
        }
        // ---------------- selection: smallest (CRC fails, metric, position)
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
        // ---------------- trace the chosen path back, one block at a time: the
        // slot it held at each block's end, then every bit from its block's word
        // (frozen bits are 0 there)
        if (lay.tg) wg_mem_order();
        else wave_mem_order();
        if (lane == 0) {
            int s = best;
            for (int jj = (N >> BL) - 1; jj >= 0; --jj) {
                chain[jj] = s;
                s = tg ? tra_g[jj * L + s] : tra_l[jj * L + s];
            }
        }
        wave_mem_order();
        const glb_ptr<uint8_t> urow_p = as_glb<uint8_t>(u_hat + urow);
        const bool aligned4 = (reinterpret_cast<uintptr_t>(u_hat + urow) & 3u) == 0;
        for (int it = 4 * lane; it < N; it += 256) {
            const int jj = it >> BL;
            const int s = chain[jj];
            const uint32_t w = (tg ? tru_g[jj * L + s] : tru_l[jj * L + s]) >> (it & (BS - 1));
            if (aligned4) {
                *(glb_ptr<uint32_t>)(urow_p + it) =
                    (w & 1u) | ((w & 2u) << 7) | ((w & 4u) << 14) | ((w & 8u) << 21);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) urow_p[it + k] = (uint8_t)((w >> k) & 1u);
            }
        }
        if (lane == 0) {
            crc_ok[f] = best_ok ? 1 : 0;
            if (pm_out) pm_out[f] = best_pm;
        }
        wave_mem_order();
    }
}

using KernelFn = void (*)(CodeDev, const float*, const int32_t*, const int32_t*, int64_t, uint8_t*, uint8_t*,
                          float*, unsigned char*, Layout, const MixedIo*);

template <int L>
KernelFn pick_bl(int bl) {
    switch (bl) {
        case 3: return &scl_kernel<L, 3>;
        case 4: return &scl_kernel<L, 4>;
        case 5: return &scl_kernel<L, 5>;
        default: return nullptr;
    }
}

// the bitonic sort is instantiated for the list sizes the comparisons use and
// threshold selection for the larger lists, both with BL = 5; the counting
// rank serves every list
KernelFn pick(int L, int n, int rank) {
    const int bl = n < 5 ? n : 5;
    if (rank == kRankBitonic && bl == 5) {
        if (L == 8) return &scl_kernel<8, 5, kRankBitonic>;
        if (L == 32) return &scl_kernel<32, 5, kRankBitonic>;
    }
    if (rank == kRankThreshold && bl == 5) {
        if (L == 8) return &scl_kernel<8, 5, kRankThreshold>;
        if (L == 16) return &scl_kernel<16, 5, kRankThreshold>;
        if (L == 32) return &scl_kernel<32, 5, kRankThreshold>;
    }
    switch (L) {
        case 1: return pick_bl<1>(bl);
        case 2: return pick_bl<2>(bl);
        case 4: return pick_bl<4>(bl);
        case 8: return pick_bl<8>(bl);
        case 16: return pick_bl<16>(bl);
        case 32: return pick_bl<32>(bl);
        default: return nullptr;
    }
}

int ps_words(int n) { return n <= 5 ? 1 : (1 << (n - 5)) - 1; }

// LDS floats per slot of the LLR heap: levels BL..gl-1 (level d at 2^d - 2^BL)
int slot_floats(int n, int gl) {
    const int bl = n < 5 ? n : 5;
    return (gl > bl ? (1 << gl) - (1 << bl) : 0) + 4;
}

// bytes of the trace: per block of 2^BL bits and path, the block's decided
// bits (32-bit word) and the slot the path held at the block start (byte)
size_t trace_bytes(int L, int N, int n) {
    const int bl = n < 5 ? n : 5;
    return (size_t)(N >> bl) * L * 5;
}

struct LdsPlan {
    size_t bytes;
    int tboff;   // LDS trace offset (tg == 0)
};

LdsPlan lds_plan(int L, int N, int n, int gl, bool tg) {
    LdsPlan p{};
    const int bl = n < 5 ? n : 5;
    size_t b = (size_t)L * slot_floats(n, gl) * 4;  // LLR heap
    b += (size_t)L * ps_words(n) * 4;                // partial sums of levels >= 5
    b += 64 * 4;                                      // candidate metrics
    // the traceback's block chain reuses the space from 0
    const size_t chain_end = align_up((size_t)(N >> bl) * 4, 16);
    b = align_up(b > chain_end ? b : chain_end, 16);
    p.tboff = 0;
    if (!tg) {
        p.tboff = (int)b;
        b += trace_bytes(L, N, n);
    }
    p.bytes = align_up(b, 16);
    return p;
}

}  // namespace scl

// candidate ranking: 0 automatic (the bitonic network for L = 8 and 32, where
// it measured fastest on MI355X; the counting rank otherwise), 1 pruned pseudo
// sort (counting), 2 bitonic network, 3 threshold selection
static std::atomic<int> g_scl_rank_mode{0};

static int rank_kind(int L) {
    switch (g_scl_rank_mode.load(std::memory_order_relaxed)) {
        case 1: return scl::kRankCount;
        case 2: return scl::kRankBitonic;
        case 3: return scl::kRankThreshold;
        default: return (L == 32 || L == 8) ? scl::kRankBitonic : scl::kRankCount;
    }
}

// LDS per workgroup; 0 (automatic) divides a CU's 160 KB among as many
// one-wave workgroups as the kernel's registers allow on a CU
static std::atomic<int64_t> g_scl_lds_budget{0};
constexpr size_t kLdsPerCu = 160 * 1024;

polar_status scl_plan(const polar_code* code, int L, int64_t max_frames, SclPlan* plan) {
    return scl_plan_dims(code->n, L, max_frames, plan);
}

polar_status scl_plan_dims(int n, int L, int64_t max_frames, SclPlan* plan) {
    const int N = 1 << n;
    scl::KernelFn fn = scl::pick(L, n, rank_kind(L));
    if (!fn) return set_error(POLAR_ERR_INVALID_ARG, "scl: L must be a power of two in [1, 32]");
    // tree levels: level 5 in LDS (read by every bit of a block), the levels
    // above in the workgroup's global slice (each written and read once per
    // block start that reaches it, as a stream); the trace in LDS if it fits
    // the budget, else in the global slice
    const int gl = n < 6 ? n : 6;
    bool tg = false;
    scl::LdsPlan lp = scl::lds_plan(L, N, n, gl, tg);
    size_t budget = (size_t)g_scl_lds_budget.load(std::memory_order_relaxed);
    if (budget == 0) {
        int by_regs = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&by_regs, fn, 64, 0) != hipSuccess || by_regs < 1) by_regs = 1;
        budget = (kLdsPerCu / (size_t)by_regs) & ~(size_t)255;
        if (budget < 4096) budget = 4096;
    }
    if (lp.bytes > budget) {
        tg = true;
        lp = scl::lds_plan(L, N, n, gl, tg);
    }
    if (lp.bytes > 160 * 1024) return set_error(POLAR_ERR_UNSUPPORTED, "scl: list too large for LDS");
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lp.bytes);
    if (e != hipSuccess || per_cu <= 0) per_cu = 1;
    int64_t grid = (int64_t)device_cu_count() * per_cu;
    if (max_frames < grid) grid = max_frames;
    if (grid < 1) grid = 1;
    plan->gl = gl;
    plan->lds_bytes = lp.bytes;
    plan->trace_glob = tg ? 1 : 0;
    plan->tb_off = lp.tboff;
    const size_t lam_b = (gl < n) ? (size_t)L * N * 4 : 0;
    plan->trace_off = lam_b;
    plan->glob_per_wg = align_up(lam_b + (tg ? scl::trace_bytes(L, N, n) : 0), 256);
    plan->grid = (int)grid;
    plan->lay_n = n;
    return POLAR_OK;
}

polar_status launch_scl(const polar_code* code, const SclPlan& plan, const float* llr, int L,
                        const int32_t* frame_ids, const int32_t* count_dev, int64_t count_host, uint8_t* u_hat,
                        uint8_t* crc_ok, float* pm, void* glob, hipStream_t stream, const MixedIo* io,
                        int64_t u_stride) {
    scl::KernelFn fn = scl::pick(L, plan.lay_n, rank_kind(L));
    scl::Layout lay;
    lay.gl = plan.gl;
    lay.sl = scl::slot_floats(plan.lay_n, plan.gl);
    lay.pw = scl::ps_words(plan.lay_n);
    lay.tg = plan.trace_glob;
    lay.nblk = (1 << plan.lay_n) >> (plan.lay_n < 5 ? plan.lay_n : 5);
    lay.gbytes = (int64_t)plan.glob_per_wg;
    lay.toff = (int64_t)plan.trace_off;
    lay.tboff = plan.tb_off;
    lay.u_stride = u_stride;
    unsigned char* gb = plan.glob_per_wg ? reinterpret_cast<unsigned char*>(glob) : nullptr;
    hipLaunchKernelGGL(fn, dim3(plan.grid), dim3(64), plan.lds_bytes, stream, code->dev(), llr, frame_ids,
                       count_dev, count_host, u_hat, crc_ok, pm, gb, lay, io);
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

extern "C" polar_status polar_set_scl_lds_budget(int64_t bytes) {
    if (bytes != 0 && (bytes < 4096 || bytes > 160 * 1024))
        return set_error(POLAR_ERR_INVALID_ARG, "polar_set_scl_lds_budget: bytes must be 0 or in [4096, 163840]");
    g_scl_lds_budget.store(bytes, std::memory_order_relaxed);
    return ok_status();
}

extern "C" int64_t polar_get_scl_lds_budget(void) { return g_scl_lds_budget.load(std::memory_order_relaxed); }

extern "C" polar_status polar_set_scl_ranking(int32_t mode) {
    if (mode < 0 || mode > 3) return set_error(POLAR_ERR_INVALID_ARG, "polar_set_scl_ranking: mode must be 0..3");
    g_scl_rank_mode.store(mode, std::memory_order_relaxed);
    return ok_status();
}

extern "C" int32_t polar_get_scl_ranking(void) { return g_scl_rank_mode.load(std::memory_order_relaxed); }
