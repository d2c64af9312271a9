// hybrid.hip -- hybrid BP -> CA-SCL decoder (Sec. III, Fig. 3).
//
// The CPU scheduling loop of Fig. 3 becomes a few kernels on one stream with
// no host round trip: BP on every frame (it writes the information bits of
// the frames it keeps), compaction of the frames whose BP verdict is not ok
// into a device queue (the failed-codeword buffer of Fig. 3), persistent CA-SCL
// workgroups that read the queue length on the device, a pass over the flags
// and statistics, and a merge of the list-decoded frames' information bits.
#include <atomic>
#include <cstring>
#include <mutex>

#include "internal.hpp"

// Device memory of hybrid_decode_batch_static: the per-batch state and the
// list decoder's global slice of one call.  Each device the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device (the name
// itself is a host-side stand-in).
static constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace polarhip {
namespace {

__global__ void clear_count_kernel(int32_t* count) {
    if (lid_x() == 0) *count = 0;
}

// queue[] <- ids of frames with ok == 0; one atomic per wavefront
__global__ __launch_bounds__(256) void compact_kernel(const uint8_t* __restrict__ ok, int64_t B,
                                                      int32_t* __restrict__ queue, int32_t* __restrict__ count) {
    const int64_t f = gid_x() * wg_size_x() + lid_x();
    const bool fail = f < B && ok[f] == 0;
    const uint64_t m = __ballot(fail);
    const int lane = __lane_id();
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(count, (int)__popcll(m));
    base = __shfl(base, 0, 64);
    if (fail) queue[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)f;
}

// used_scl and the statistics of every frame, reduced per wavefront before
// the atomics (the information bits of the frames BP kept were written by the
// BP kernel)
__global__ __launch_bounds__(256) void flags_kernel(const uint8_t* __restrict__ ok,
                                                    const int32_t* __restrict__ iters, int64_t B,
                                                    uint8_t* __restrict__ used_scl,
                                                    unsigned long long* __restrict__ stats) {
    const int64_t f = gid_x() * 256 + lid_x();
    unsigned long long s_n = 0, s_bp = 0, s_scl = 0, s_it = 0;
    if (f < B) {
        const bool good = ok[f] != 0;
        if (used_scl) used_scl[f] = good ? 0 : 1;
        s_n = 1;
        s_bp = good;
        s_scl = !good;
        s_it = (unsigned long long)iters[f];
    }
    if (stats) {
        for (int m = 32; m >= 1; m >>= 1) {
            s_n += __shfl_xor(s_n, m, 64);
            s_bp += __shfl_xor(s_bp, m, 64);
            s_scl += __shfl_xor(s_scl, m, 64);
            s_it += __shfl_xor(s_it, m, 64);
        }
        if ((lid_x() & 63) == 0 && s_n) {
            atomicAdd(&stats[0], s_n);
            if (s_bp) atomicAdd(&stats[1], s_bp);
            if (s_scl) atomicAdd(&stats[2], s_scl);
            atomicAdd(&stats[3], s_it);
        }
    }
}

// information bits of the list-decoded frames queue[0 .. *count), one
// workgroup per frame (persistent over the count on the device), and the
// count of those whose CRC failed
__global__ __launch_bounds__(256) void merge_scl_kernel(CodeDev code, const uint8_t* __restrict__ u_hat,
                                                        const int32_t* __restrict__ queue,
                                                        const int32_t* __restrict__ count,
                                                        const uint8_t* __restrict__ scl_ok,
                                                        uint8_t* __restrict__ info_hat,
                                                        unsigned long long* __restrict__ stats) {
    const int K = code.K, N = code.N;
    const int64_t cnt = *count;
    for (int64_t i = gid_x(); i < cnt; i += num_groups_x()) {
        const int64_t f = queue[i];
        for (int q = lid_x(); q < K; q += 256) info_hat[f * K + q] = u_hat[f * N + code.info_pos[q]];
        if (lid_x() == 0 && stats && !scl_ok[f]) atomicAdd(&stats[4], 1ull);
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

// per-batch state of B frames from `off`; returns the end offset
size_t carve_batch(const polar_code* code, int64_t B, size_t off, char* base, HybridWs* w) {
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
    if (base) {
        w->u_hat = reinterpret_cast<uint8_t*>(base + o_u);
        w->ok = reinterpret_cast<uint8_t*>(base + o_ok);
        w->iters = reinterpret_cast<int32_t*>(base + o_it);
        w->queue = reinterpret_cast<int32_t*>(base + o_q);
        w->count = reinterpret_cast<int32_t*>(base + o_c);
        w->scl_ok = reinterpret_cast<uint8_t*>(base + o_s);
    }
    return off;
}

// `slots` copies of the per-batch state followed by one list-decoder slice
size_t carve(const polar_code* code, int64_t B, const SclPlan& plan, void* base, HybridWs* w, int slots) {
    char* b = static_cast<char*>(base);
    size_t off = 0;
    for (int s = 0; s < slots; ++s) off = carve_batch(code, B, off, b, w ? &w[s] : nullptr);
    const size_t o_g = off;
    off = align_up(off + plan.glob_per_wg * plan.grid, 256);
    if (b && w)
        for (int s = 0; s < slots; ++s) {
            w[s].scl_glob = plan.glob_per_wg ? (void*)(b + o_g) : nullptr;
            w[s].total = off;
        }
    return off;
}

// BP and list-decoder workgroups per CU in the pipelined hybrid (0: no limit)
std::atomic<int> g_pipe_bp_wgs{0};
std::atomic<int> g_pipe_scl_wgs{0};

// per-batch states in flight in the pipelined hybrid: batch j + kPipeSlots
// reuses batch j's state, so its BP waits for batch j's merge (three states
// measured no faster than two: the list decoder and the next BP compete for
// the same CUs, not for the state)
constexpr int kPipeSlots = 2;

// the events (BP done and SCL done, per slot) of the calling thread on the
// current device, created on first use and kept: a later call re-records them
// after every wait that an earlier call enqueued on them
polar_status pipeline_events(hipEvent_t** out) {
    constexpr int kMaxDev = 64;
    thread_local hipEvent_t ev[kMaxDev][2 * kPipeSlots] = {};
    int dev = 0;
    polar_status st = hip_check(hipGetDevice(&dev), "get device");
    if (st != POLAR_OK) return st;
    if (dev < 0 || dev >= kMaxDev) return set_error(POLAR_ERR_UNSUPPORTED, "device index out of range");
    for (int i = 0; i < 2 * kPipeSlots; ++i)
        if (!ev[dev][i] &&
            (st = hip_check(hipEventCreateWithFlags(&ev[dev][i], hipEventDisableTiming), "event create")) != POLAR_OK)
            return st;
    *out = ev[dev];
    return POLAR_OK;
}

// BP (writing the information bits of the frames it keeps straight to
// info_hat) and compaction of one batch on `stream`
polar_status enqueue_bp_part(const polar_code* code, const float* llr, int64_t B, const bp_params* p,
                             const HybridWs& w, uint8_t* info_hat, hipStream_t stream, int wgs_per_cu = 0) {
    polar_status st = launch_bp(code, llr, B, p, nullptr, nullptr, w.iters, w.ok, stream, wgs_per_cu, info_hat);
    if (st != POLAR_OK) return st;
    hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(64), 0, stream, w.count);
    const unsigned cblocks = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(compact_kernel, dim3(cblocks), dim3(256), 0, stream, w.ok, B, w.queue, w.count);
    return hip_check(hipGetLastError(), "compact launch");
}

// CA-SCL on the queued frames and the merge, on `stream`
polar_status enqueue_scl_part(const polar_code* code, const SclPlan& plan, const float* llr, int64_t B, int L,
                              const HybridWs& w, uint8_t* info_hat, uint8_t* used_scl, int64_t* stats,
                              hipStream_t stream) {
    polar_status st = launch_scl(code, plan, llr, L, w.queue, w.count, 0, w.u_hat, w.scl_ok, nullptr, w.scl_glob,
                                 stream);
    if (st != POLAR_OK) return st;
    unsigned long long* st64 = reinterpret_cast<unsigned long long*>(stats);
    hipLaunchKernelGGL(flags_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, w.ok, w.iters, B,
                       used_scl, st64);
    const int64_t mgrid = B < 4096 ? B : 4096;
    hipLaunchKernelGGL(merge_scl_kernel, dim3((unsigned)mgrid), dim3(256), 0, stream, code->dev(), w.u_hat, w.queue,
                       w.count, w.scl_ok, info_hat, st64);
    return hip_check(hipGetLastError(), "merge launch");
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

static polar_status check_bp_params(const polar_code* code, const bp_params* p) {
    if (p->max_iter < 1) return set_error(POLAR_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (p->stop < 0 || p->stop > 2) return set_error(POLAR_ERR_INVALID_ARG, "stop must be 0, 1 or 2");
    if (p->stop == 2 && code->c == 0) return set_error(POLAR_ERR_INVALID_ARG, "CRC stop needs a code with a CRC");
    if (!(p->llr_max > 0.0f)) return set_error(POLAR_ERR_INVALID_ARG, "llr_max must be > 0");
    if (p->rule != 0 && p->rule != 1) return set_error(POLAR_ERR_INVALID_ARG, "rule must be 0 or 1");
    if (p->rule == 1 && p->weights) return set_error(POLAR_ERR_UNSUPPORTED, "the exact rule has no weighted form");
    if (p->weights && p->weight_iters < p->max_iter) return set_error(POLAR_ERR_INVALID_ARG, "weight_iters < max_iter");
    if (p->weight_layout != 0 && p->weight_layout != 1) return set_error(POLAR_ERR_INVALID_ARG, "weight_layout must be 0 or 1");
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
    *bytes = params ? carve(code, B, plan, nullptr, nullptr, 1) : plan.glob_per_wg * plan.grid;
    return ok_status();
}

extern "C" polar_status polar_pipeline_workspace_size(const polar_code* code, int64_t B, int32_t L,
                                                      const bp_params* params, size_t* bytes) {
    if (!code || !bytes || !params || B < 0)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_pipeline_workspace_size: bad argument");
    SclPlan plan;
    polar_status st = scl_plan(code, L, B > 0 ? B : 1, &plan);
    if (st != POLAR_OK) return st;
    *bytes = carve(code, B, plan, nullptr, nullptr, kPipeSlots);
    return ok_status();
}

namespace {

// Captured graphs of hybrid_decode_batch.  A call's work is fully determined
// by this key (the kernels read the weights, LLRs and tables through the
// pointers, so their contents may change between calls); the first call with
// a key runs the kernels directly, the second captures them into a graph on a
// library stream and every later one replays that graph on the caller's
// stream.  Codes carry a serial number, so a code freed and another built at
// the same address never match.
struct HybridKey {
    int dev;
    const polar_code* code;
    uint64_t serial;
    const float* llr;
    int64_t B;
    bp_params p;
    int32_t L;
    uint8_t* info_hat;
    uint8_t* used_scl;
    int64_t* stats;
    void* ws;
    int64_t lds_budget;
    int32_t ranking;
    bool operator==(const HybridKey& o) const {
        return dev == o.dev && code == o.code && serial == o.serial && llr == o.llr && B == o.B &&
               p.max_iter == o.p.max_iter && p.stop == o.p.stop && p.llr_max == o.p.llr_max &&
               p.rule == o.p.rule && p.weights == o.p.weights && p.weight_iters == o.p.weight_iters &&
               p.variant == o.p.variant && p.weight_layout == o.p.weight_layout && L == o.L &&
               info_hat == o.info_hat && used_scl == o.used_scl && stats == o.stats && ws == o.ws &&
               lds_budget == o.lds_budget && ranking == o.ranking;
    }
};

struct HybridGraph {
    HybridKey key;
    int calls = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;  // last use, for replacement
};

constexpr int kGraphSlots = 8;
std::mutex g_graph_mu;
HybridGraph g_graphs[kGraphSlots];
uint64_t g_graph_clock = 0;
std::atomic<int> g_graph_mode{1};

// per-device stream on which hybrid graphs are captured
polar_status capture_stream(int dev, hipStream_t* out) {
    constexpr int kMaxDev = 64;
    static hipStream_t streams[kMaxDev] = {};
    if (dev < 0 || dev >= kMaxDev) return set_error(POLAR_ERR_UNSUPPORTED, "device index out of range");
    if (!streams[dev]) {
        polar_status st = hip_check(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking), "stream create");
        if (st != POLAR_OK) return st;
    }
    *out = streams[dev];
    return POLAR_OK;
}

polar_status enqueue_hybrid(const polar_code* code, const SclPlan& plan, const float* llr, int64_t B,
                            const bp_params* p, int32_t L, uint8_t* info_hat, uint8_t* used_scl, int64_t* stats,
                            void* ws, hipStream_t stream) {
    HybridWs w;
    carve(code, B, plan, ws, &w, 1);
    polar_status st = enqueue_bp_part(code, llr, B, p, w, info_hat, stream);
    if (st != POLAR_OK) return st;
    return enqueue_scl_part(code, plan, llr, B, L, w, info_hat, used_scl, stats, stream);
}

}  // namespace

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
    const size_t need = carve(code, B, plan, nullptr, nullptr, 1);
    if (!ws || ws_bytes < need) return set_error(POLAR_ERR_WORKSPACE, "hybrid_decode_batch: workspace too small");
    if (B == 0) return ok_status();
    // work enqueued on a stream the caller is capturing is recorded there
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if ((st = hip_check(hipStreamIsCapturing(stream, &cap), "stream capture query")) != POLAR_OK) return st;
    if (g_graph_mode.load() == 0 || cap != hipStreamCaptureStatusNone) {
        st = enqueue_hybrid(code, plan, llr, B, p, L, info_hat, used_scl, stats, ws, stream);
        return st == POLAR_OK ? ok_status() : st;
    }
    HybridKey key;
    std::memset(&key, 0, sizeof(key));
    if ((st = hip_check(hipGetDevice(&key.dev), "get device")) != POLAR_OK) return st;
    key.code = code;
    key.serial = code->serial;
    key.llr = llr;
    key.B = B;
    key.p = *p;
    key.L = L;
    key.info_hat = info_hat;
    key.used_scl = used_scl;
    key.stats = stats;
    key.ws = ws;
    key.lds_budget = polar_get_scl_lds_budget();
    key.ranking = polar_get_scl_ranking();
    std::lock_guard<std::mutex> lock(g_graph_mu);
    HybridGraph* slot = nullptr;
    for (HybridGraph& g : g_graphs)
        if (g.calls > 0 && g.key == key) slot = &g;
    if (!slot) {
        // first call with this key: run directly and remember the key in the
        // least recently used slot
        HybridGraph* victim = &g_graphs[0];
        for (HybridGraph& g : g_graphs)
            if (g.used < victim->used) victim = &g;
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        if (victim->graph) (void)hipGraphDestroy(victim->graph);
        *victim = HybridGraph();
        victim->key = key;
        victim->calls = 1;
        victim->used = ++g_graph_clock;
        st = enqueue_hybrid(code, plan, llr, B, p, L, info_hat, used_scl, stats, ws, stream);
        return st == POLAR_OK ? ok_status() : st;
    }
    slot->used = ++g_graph_clock;
    if (!slot->exec) {
        hipStream_t cs = nullptr;
        if ((st = capture_stream(key.dev, &cs)) != POLAR_OK) return st;
        if ((st = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) != POLAR_OK)
            return st;
        polar_status se = enqueue_hybrid(code, plan, llr, B, p, L, info_hat, used_scl, stats, ws, cs);
        hipGraph_t g = nullptr;
        st = hip_check(hipStreamEndCapture(cs, &g), "end capture");
        if (se != POLAR_OK || st != POLAR_OK) {
            if (g) (void)hipGraphDestroy(g);
            return se != POLAR_OK ? se : st;
        }
        hipGraphExec_t ex = nullptr;
        if ((st = hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate")) != POLAR_OK) {
            (void)hipGraphDestroy(g);
            return st;
        }
        slot->graph = g;
        slot->exec = ex;
    }
    ++slot->calls;
    st = hip_check(hipGraphLaunch(slot->exec, stream), "graph launch");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status polar_set_hybrid_graphs(int32_t mode) {
    if (mode != 0 && mode != 1) return set_error(POLAR_ERR_INVALID_ARG, "polar_set_hybrid_graphs: mode must be 0 or 1");
    g_graph_mode.store(mode);
    return ok_status();
}

extern "C" int32_t polar_get_hybrid_graphs(void) { return g_graph_mode.load(); }

// device address of `scratch` on the current device, looked up once per device
static polar_status static_scratch(void** out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static void* addr[kMaxDev] = {};
    int dev = 0;
    polar_status st = hip_check(hipGetDevice(&dev), "get device");
    if (st != POLAR_OK) return st;
    if (dev < 0 || dev >= kMaxDev) return set_error(POLAR_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (st != POLAR_OK) return st;
        if (!p) return set_error(POLAR_ERR_DEVICE, "scratch symbol address is null");
        addr[dev] = p;
    }
    *out = addr[dev];
    return POLAR_OK;
}

extern "C" polar_status hybrid_decode_batch_static(const polar_code* code, const float* llr, int64_t B,
                                                   const bp_params* p, int32_t L, uint8_t* info_hat,
                                                   uint8_t* used_scl, int64_t* stats, hipStream_t stream) {
    if (!code || !p) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch_static: null code or params");
    if (B < 0 || B > (int64_t)INT32_MAX)
        return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch_static: bad batch size");
    if (B > 0 && (!llr || !info_hat))
        return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch_static: null buffer");
    polar_status st = check_bp_params(code, p);
    if (st != POLAR_OK) return st;
    SclPlan plan;
    if ((st = scl_plan(code, L, B > 0 ? B : 1, &plan)) != POLAR_OK) return st;
    // the per-batch state first; the list decoder then runs as many
    // persistent workgroups as global slices fit in the rest (at least one)
    const size_t batch = carve_batch(code, B, 0, nullptr, nullptr);
    if (batch + plan.glob_per_wg > kStaticScratchBytes)
        return set_error(POLAR_ERR_INVALID_ARG,
                         "hybrid_decode_batch_static: batch needs " + std::to_string(batch + plan.glob_per_wg) +
                             " bytes of scratch, the maximum is " + std::to_string(kStaticScratchBytes));
    if (plan.glob_per_wg) {
        const size_t fit = (kStaticScratchBytes - batch) / plan.glob_per_wg;
        if ((size_t)plan.grid > fit) plan.grid = (int)fit;
    }
    if (carve(code, B, plan, nullptr, nullptr, 1) > kStaticScratchBytes)
        return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_batch_static: batch too large for the scratch");
    if (B == 0) return ok_status();
    void* ws = nullptr;
    if ((st = static_scratch(&ws)) != POLAR_OK) return st;
    HybridWs w;
    carve(code, B, plan, ws, &w, 1);
    if ((st = enqueue_bp_part(code, llr, B, p, w, info_hat, stream)) != POLAR_OK) return st;
    if ((st = enqueue_scl_part(code, plan, llr, B, L, w, info_hat, used_scl, stats, stream)) != POLAR_OK) return st;
    return ok_status();
}

extern "C" polar_status hybrid_decode_pipelined(const polar_code* code, int64_t nbatch, const float* const* llr,
                                                int64_t B, const bp_params* p, int32_t L, uint8_t* const* info_hat,
                                                uint8_t* const* used_scl, int64_t* stats, void* ws, size_t ws_bytes,
                                                hipStream_t stream_bp, hipStream_t stream_scl) {
    if (!code || !p) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_pipelined: null code or params");
    if (nbatch < 0 || B < 0 || B > (int64_t)INT32_MAX)
        return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_pipelined: bad batch count or size");
    if (stream_bp == stream_scl) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_pipelined: streams must differ");
    if (nbatch > 0 && B > 0) {
        if (!llr || !info_hat) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_pipelined: null pointer array");
        for (int64_t j = 0; j < nbatch; ++j)
            if (!llr[j] || !info_hat[j]) return set_error(POLAR_ERR_INVALID_ARG, "hybrid_decode_pipelined: null buffer");
    }
    polar_status st = check_bp_params(code, p);
    if (st != POLAR_OK) return st;
    SclPlan plan;
    if ((st = scl_plan(code, L, B > 0 ? B : 1, &plan)) != POLAR_OK) return st;
    // fewer persistent list-decoder workgroups (each walks more of the queue)
    // use fewer global slices, so the workspace size query stays an upper bound
    if (const int cap_wgs = g_pipe_scl_wgs.load(); cap_wgs > 0) {
        const int64_t cap = (int64_t)device_cu_count() * cap_wgs;
        if (plan.grid > cap) plan.grid = (int)(cap > 0 ? cap : 1);
    }
    const size_t need = carve(code, B, plan, nullptr, nullptr, kPipeSlots);
    if (!ws || ws_bytes < need) return set_error(POLAR_ERR_WORKSPACE, "hybrid_decode_pipelined: workspace too small");
    if (nbatch == 0 || B == 0) return ok_status();
    HybridWs w[kPipeSlots];
    carve(code, B, plan, ws, w, kPipeSlots);
    hipEvent_t* ev = nullptr;
    if ((st = pipeline_events(&ev)) != POLAR_OK) return st;
    hipEvent_t* bp_done = ev;
    hipEvent_t* scl_done = ev + kPipeSlots;
    // the first batches must not start before work already queued on stream_scl
    // has finished with the shared list-decoder slice of an earlier call
    if (st == POLAR_OK) st = hip_check(hipEventRecord(scl_done[0], stream_scl), "event record");
    if (st == POLAR_OK) st = hip_check(hipStreamWaitEvent(stream_bp, scl_done[0], 0), "stream wait");
    for (int64_t j = 0; j < nbatch && st == POLAR_OK; ++j) {
        const int s = (int)(j % kPipeSlots);
        if (j >= kPipeSlots) st = hip_check(hipStreamWaitEvent(stream_bp, scl_done[s], 0), "stream wait");
        if (st == POLAR_OK) st = enqueue_bp_part(code, llr[j], B, p, w[s], info_hat[j], stream_bp, g_pipe_bp_wgs.load());
        if (st == POLAR_OK) st = hip_check(hipEventRecord(bp_done[s], stream_bp), "event record");
        if (st == POLAR_OK) st = hip_check(hipStreamWaitEvent(stream_scl, bp_done[s], 0), "stream wait");
        if (st == POLAR_OK)
            st = enqueue_scl_part(code, plan, llr[j], B, L, w[s], info_hat[j], used_scl ? used_scl[j] : nullptr,
                                  stats, stream_scl);
        if (st == POLAR_OK) st = hip_check(hipEventRecord(scl_done[s], stream_scl), "event record");
    }
    if (st == POLAR_OK)
        st = hip_check(hipStreamWaitEvent(stream_bp, scl_done[(int)((nbatch - 1) % kPipeSlots)], 0), "stream wait");
    return st == POLAR_OK ? ok_status() : st;
}

extern "C" polar_status polar_set_pipeline_bp_occupancy(int32_t wgs_per_cu) {
    if (wgs_per_cu < 0 || wgs_per_cu > 64)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_set_pipeline_bp_occupancy: must be in [0, 64]");
    g_pipe_bp_wgs.store(wgs_per_cu);
    return ok_status();
}

extern "C" int32_t polar_get_pipeline_bp_occupancy(void) { return g_pipe_bp_wgs.load(); }

extern "C" polar_status polar_set_pipeline_scl_occupancy(int32_t wgs_per_cu) {
    if (wgs_per_cu < 0 || wgs_per_cu > 64)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_set_pipeline_scl_occupancy: must be in [0, 64]");
    g_pipe_scl_wgs.store(wgs_per_cu);
    return ok_status();
}

extern "C" int32_t polar_get_pipeline_scl_occupancy(void) { return g_pipe_scl_wgs.load(); }
