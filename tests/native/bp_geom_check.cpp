// Host-side verification of the BP kernel's compile-time data layout
// (paper_1609_09358_amd/csrc/bp_geom.hpp), run before any GPU launch:
//   - windows cover every PE column once, each column's pair bit is a
//     register bit of its window, node_index is a bijection per window;
//   - every LDS transpose (both directions, every boundary) stays inside the
//     buffer, never lets two values share a word, and reads back exactly the
//     node that was written;
//   - the 32 lanes of every half-wavefront hit 32 distinct banks on both sides;
//   - wavefronts never share words in the barrier-free (intra-wave) buffer,
//     and the buffers of different barrier-separated transposes are disjoint.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../../paper_1609_09358_amd/csrc/bp_geom.hpp"

using namespace polarhip::bp;

static int failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            ++failures;                                    \
            if (failures < 30) {                           \
                std::printf("FAIL n=%d r=%d: ", G::n, G::r); \
                std::printf(__VA_ARGS__);                  \
                std::printf("\n");                         \
            }                                              \
        }                                                  \
    } while (0)

template <int NL, int RL>
void check() {
    using G = Geom<NL, RL>;
    // windows
    std::vector<int> cover(G::n, 0);
    for (int k = 0; k < G::NWIN; ++k)
        for (int s = G::cbeg(k); s < G::cend(k); ++s) {
            cover[s]++;
            int q = s - G::wbase(k);
            CHECK(q >= 0 && q < G::r, "column %d not a register bit of window %d", s, k);
        }
    for (int s = 0; s < G::n; ++s) CHECK(cover[s] == 1, "column %d covered %d times", s, cover[s]);
    for (int k = 0; k < G::NWIN; ++k) {
        std::vector<int> seen(G::N, 0);
        for (int t = 0; t < G::T; ++t)
            for (int v = 0; v < G::V; ++v) {
                int i = node_index<G>(k, t, v);
                CHECK(i >= 0 && i < G::N, "index out of range");
                if (i >= 0 && i < G::N) seen[i]++;
            }
        for (int i = 0; i < G::N; ++i) CHECK(seen[i] == 1, "window %d node %d held %d times", k, i, seen[i]);
    }
    CHECK(G::wbase(0) == 0, "window 0 must hold the low bits");
    // transposes
    std::vector<std::set<int>> wave_words(G::NWAVES);
    for (int j = 0; j < G::NB; ++j) {
        const auto& B = G::TAB.b[j];
        for (int dir = 0; dir < 2; ++dir) {
            const bool is_r = dir == 0;
            const int kf = is_r ? j : j + 1, kt = is_r ? j + 1 : j;
            std::vector<long> mem(G::TAB.words, -1);
            const int base = is_r ? B.buf_r : B.buf_l;
            for (int tid = 0; tid < G::WG; ++tid) {
                int t = G::T < 64 ? (tid & (G::T - 1)) : tid;
                int slot = G::T < 64 ? (tid >> G::P) : 0;
                for (int v = 0; v < G::V; ++v) {
                    int a = lds_word<G>(j, kf, t, slot, v, is_r);
                    CHECK(a >= base && a < base + B.size && a < G::TAB.words, "bnd %d write out of range %d", j, a);
                    if (a < 0 || a >= G::TAB.words) continue;
                    CHECK(mem[a] == -1, "bnd %d dir %d word %d written twice", j, dir, a);
                    mem[a] = (long)slot * G::N + node_index<G>(kf, t, v);
                    if (!B.cross) wave_words[tid / 64].insert(a);
                }
            }
            for (int tid = 0; tid < G::WG; ++tid) {
                int t = G::T < 64 ? (tid & (G::T - 1)) : tid;
                int slot = G::T < 64 ? (tid >> G::P) : 0;
                for (int v = 0; v < G::V; ++v) {
                    int a = lds_word<G>(j, kt, t, slot, v, is_r);
                    if (a < 0 || a >= G::TAB.words) {
                        CHECK(false, "read out of range");
                        continue;
                    }
                    long want = (long)slot * G::N + node_index<G>(kt, t, v);
                    CHECK(mem[a] == want, "bnd %d dir %d: read %ld want %ld", j, dir, mem[a], want);
                    if (!B.cross) wave_words[tid / 64].insert(a);
                }
            }
            // bank conflicts per half-wavefront and register
            for (int side = 0; side < 2; ++side) {
                int k = side ? kt : kf;
                for (int h0 = 0; h0 < G::WG; h0 += 32)
                    for (int v = 0; v < G::V; ++v) {
                        std::set<int> banks;
                        for (int l = 0; l < 32; ++l) {
                            int tid = h0 + l;
                            int t = G::T < 64 ? (tid & (G::T - 1)) : tid;
                            int slot = G::T < 64 ? (tid >> G::P) : 0;
                            banks.insert(lds_word<G>(j, k, t, slot, v, is_r) % 32);
                        }
                        CHECK((int)banks.size() == 32, "bnd %d dir %d side %d: %zu banks", j, dir, side, banks.size());
                    }
            }
        }
    }
    // intra buffer: wavefronts disjoint; cross buffers disjoint from everything
    for (int a = 0; a < G::NWAVES; ++a)
        for (int b = a + 1; b < G::NWAVES; ++b)
            for (int w : wave_words[a]) CHECK(!wave_words[b].count(w), "waves %d,%d share word %d", a, b, w);
    std::vector<std::pair<int, int>> ranges;
    int intra_end = 0;
    for (int j = 0; j < G::NB; ++j) {
        const auto& B = G::TAB.b[j];
        if (B.cross) {
            ranges.push_back({B.buf_r, B.buf_r + B.size});
            ranges.push_back({B.buf_l, B.buf_l + B.size});
        } else {
            intra_end = B.size > intra_end ? B.size : intra_end;
        }
    }
    if (intra_end) ranges.push_back({0, intra_end});
    for (size_t a = 0; a < ranges.size(); ++a)
        for (size_t b = a + 1; b < ranges.size(); ++b)
            CHECK(ranges[a].second <= ranges[b].first || ranges[b].second <= ranges[a].first, "buffers overlap");
    // a barrier-free frame must have a cross boundary when it spans wavefronts
    bool any_cross = false;
    for (int j = 0; j < G::NB; ++j) any_cross = any_cross || G::TAB.b[j].cross;
    CHECK(G::NWAVES == 1 || any_cross, "multi-wave frame without a barrier-separated boundary");
    std::printf("n=%2d r=%d T=%4d FPW=%2d windows=%d words=%6d (%.3f of FPW*N) cross=%d\n", G::n, G::r, G::T, G::FPW,
                G::NWIN, G::TAB.words, double(G::TAB.words) / (G::FPW * G::N), (int)any_cross);
}

template <int NL>
void both() {
    check<NL, 2>();
    check<NL, 3>();
}

int main() {
    both<3>();
    both<4>();
    both<5>();
    both<6>();
    both<7>();
    both<8>();
    both<9>();
    both<10>();
    both<11>();
    both<12>();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("all layouts verified\n");
    return 0;
}
