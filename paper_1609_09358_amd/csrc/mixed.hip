// mixed.hip -- hybrid decoding of ragged batches that mix several codes
// (block lengths and rates), as one device pipeline or one replayed hipGraph.
//
// A call: a one-thread kernel stores the call's arguments in a device block;
// counters are cleared by a kernel (no memset node, so the pipeline can be
// captured); a bucketing kernel appends every frame id to the list of its
// block length; then, per block length, as concurrent branches on the plan's
// streams: a persistent BP kernel walks the list (its length read on the
// device) decoding every frame with its own code and appends the frames whose
// verdict is not ok to the group's queue, and a persistent CA-SCL kernel
// drains that queue, again with each frame's own code (its layout holds the
// group's largest block length).  After the branches join, a merge kernel
// writes every frame's information bits, its list-decoder flag and the
// statistics.  (Codes shorter than 32 bits form one group each.)  No host round trip and no per-call
// allocation: the plan owns its workspace.  Because the kernels read the
// per-call buffers through the argument block, the same captured graph
// serves every call.
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace polarhip {
namespace {

constexpr int kMaxCodes = 16;
constexpr int kMaxBranches = 4;

struct MixedArgs {
    MixedIo io;                    // llr, llr_off
    int64_t B;
    const int32_t* code_of_frame;  // [B]
    const int64_t* out_off;        // [B]
    uint8_t* info_hat;
    uint8_t* used_scl;             // [B] or null
    int64_t* stats;                // [8] or null
};

__global__ void set_args_kernel(MixedArgs* d, MixedArgs v) {
    if (lid_x() == 0) *d = v;
}

__global__ void clear_kernel(int32_t* c, int n) {
    if ((int)lid_x() < n) c[lid_x()] = 0;
}

// ids of group g (the group of the frame's code): lists[g * cap + ...], cnt[g] of them
__global__ __launch_bounds__(256) void bucket_kernel(const MixedArgs* __restrict__ a, int n_codes, int64_t cap,
                                                     const int32_t* __restrict__ group_of_code,
                                                     int32_t* __restrict__ lists, int32_t* __restrict__ cnt) {
    const int64_t f = gid_x() * wg_size_x() + lid_x();
    if (f >= a->B || f >= cap) return;
    const int c = a->code_of_frame[f];
    if (c < 0 || c >= n_codes) return;
    const int g = group_of_code[c];
    lists[(int64_t)g * cap + atomicAdd(&cnt[g], 1)] = (int32_t)f;
}

// one wavefront per frame
__global__ __launch_bounds__(64) void mixed_merge_kernel(const MixedArgs* __restrict__ a, const CodeDev* __restrict__ codes,
                                                         int n_codes, const uint8_t* __restrict__ u, int64_t u_stride,
                                                         const uint8_t* __restrict__ ok,
                                                         const int32_t* __restrict__ iters,
                                                         const uint8_t* __restrict__ scl_ok) {
    const int64_t f = gid_x();
    if (f >= a->B) return;
    const int c = a->code_of_frame[f];
    if (c < 0 || c >= n_codes) return;
    const CodeDev& cd = codes[c];
    const uint8_t* uf = u + f * u_stride;
    uint8_t* dst = a->info_hat + a->out_off[f];
    for (int q = lid_x(); q < cd.K; q += 64) dst[q] = uf[cd.info_pos[q]];
    if (lid_x() == 0) {
        const bool good = ok[f] != 0;
        if (a->used_scl) a->used_scl[f] = good ? 0 : 1;
        if (a->stats) {
            unsigned long long* st = reinterpret_cast<unsigned long long*>(a->stats);
            atomicAdd(&st[0], 1ull);
            if (good) atomicAdd(&st[1], 1ull);
            else atomicAdd(&st[2], 1ull);
            atomicAdd(&st[3], (unsigned long long)iters[f]);
            if (!good && !scl_ok[f]) atomicAdd(&st[4], 1ull);
        }
    }
}

}  // namespace
}  // namespace polarhip

using namespace polarhip;

struct polar_mixed {
    int device = 0;
    int n_codes = 0;
    int64_t cap = 0;  // max frames per call
    int L = 0;
    int maxN = 0;
    std::vector<const polar_code*> codes;
    // groups: codes of one block length (one code each below 32 bits)
    int n_groups = 0;
    std::vector<int> rep;           // per group: its first code
    std::vector<bp_params> params;  // per group (the first code's variant)
    std::vector<SclPlan> scl;       // per group
    std::vector<int> bp_grid;       // per group
    // device memory (one allocation)
    void* mem = nullptr;
    MixedArgs* dargs = nullptr;
    CodeDev* dcodes = nullptr;
    int32_t* gmap = nullptr;    // [n_codes] group of each code
    int32_t* counts = nullptr;  // [2 * n_codes]: bucket sizes, then queue sizes
    int32_t* lists = nullptr;   // [n_groups][cap]
    int32_t* queues = nullptr;  // [n_groups][cap]
    uint8_t* ok = nullptr;
    int32_t* iters = nullptr;
    uint8_t* scl_ok = nullptr;
    uint8_t* u = nullptr;  // [cap][maxN]
    std::vector<void*> glob;  // per list-decoder launch: its global slice
    int nbr = 0;
    hipStream_t br[kMaxBranches] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kMaxBranches] = {};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void mixed_release(polar_mixed* m) {
    if (!m) return;
    if (m->exec) hipGraphExecDestroy(m->exec);
    if (m->graph) hipGraphDestroy(m->graph);
    for (int s = 0; s < m->nbr; ++s) {
        if (m->ev_join[s]) hipEventDestroy(m->ev_join[s]);
        if (m->br[s]) hipStreamDestroy(m->br[s]);
    }
    if (m->ev_fork) hipEventDestroy(m->ev_fork);
    if (m->cap_stream) hipStreamDestroy(m->cap_stream);
    if (m->mem) hipFree(m->mem);
    delete m;
}

extern "C" polar_status polar_mixed_create(const polar_code* const* codes, int32_t n_codes, int64_t max_frames,
                                           const bp_params* params, int32_t L, const int32_t* variants,
                                           polar_mixed** out) {
    if (!out || !codes || !params) return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: null argument");
    *out = nullptr;
    if (n_codes < 1 || n_codes > kMaxCodes)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: n_codes must be in [1, 16]");
    if (max_frames < 1 || max_frames > (int64_t)INT32_MAX)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: max_frames must be in [1, 2^31)");
    if (params->weights) return set_error(POLAR_ERR_UNSUPPORTED, "polar_mixed_create: weighted BP is per code");
    if (params->max_iter < 1 || params->stop < 0 || params->stop > 2 || !(params->llr_max > 0.0f) || params->rule != 0)
        return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: bad BP parameters");
    int dev = 0;
    polar_status st = hip_check(hipGetDevice(&dev), "get device");
    if (st != POLAR_OK) return st;
    polar_mixed* m = new polar_mixed();
    m->device = dev;
    m->n_codes = n_codes;
    m->cap = max_frames;
    m->L = L;
    for (int c = 0; c < n_codes; ++c) {
        const polar_code* code = codes[c];
        if (!code || code->device != dev) {
            mixed_release(m);
            return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: null code or code of another device");
        }
        if (params->stop == 2 && code->c == 0) {
            mixed_release(m);
            return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: CRC stop needs codes with a CRC");
        }
        const int v = variants ? variants[c] : 0;
        if (v != 0 && !bp_variant_supported(code->n, v)) {
            mixed_release(m);
            return set_error(POLAR_ERR_INVALID_ARG, "polar_mixed_create: unknown BP variant");
        }
        m->codes.push_back(code);
        if (code->N > m->maxN) m->maxN = code->N;
    }
    // groups: one per block length (one BP kernel and one list-decoder kernel
    // serve the group's codes); a code shorter than 32 bits forms its own
    std::vector<int32_t> gmap(n_codes);
    for (int c = 0; c < n_codes; ++c) {
        int g = -1;
        if (codes[c]->n >= 5)
            for (int h = 0; h < m->n_groups; ++h)
                if (codes[m->rep[h]]->N == codes[c]->N) g = h;
        if (g < 0) {
            g = m->n_groups++;
            m->rep.push_back(c);
        }
        gmap[c] = g;
    }
    for (int g = 0; g < m->n_groups; ++g) {
        const int c = m->rep[g];
        bp_params p = *params;
        p.variant = variants ? variants[c] : 0;
        int grid = 0;
        SclPlan sp;
        if ((st = bp_gather_grid(codes[c], &p, max_frames, &grid)) != POLAR_OK ||
            (st = scl_plan_dims(codes[c]->n, L, max_frames, &sp)) != POLAR_OK) {
            mixed_release(m);
            return st;
        }
        m->params.push_back(p);
        m->bp_grid.push_back(grid);
        m->scl.push_back(sp);
    }
    // one device allocation, carved
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_args = take(sizeof(MixedArgs));
    const size_t o_codes = take(sizeof(CodeDev) * n_codes);
    const size_t o_gmap = take(sizeof(int32_t) * n_codes);
    const size_t o_cnt = take(sizeof(int32_t) * 2 * n_codes);
    const size_t o_lists = take(sizeof(int32_t) * m->n_groups * max_frames);
    const size_t o_queues = take(sizeof(int32_t) * m->n_groups * max_frames);
    const size_t o_ok = take(max_frames);
    const size_t o_it = take(sizeof(int32_t) * max_frames);
    const size_t o_sok = take(max_frames);
    const size_t o_u = take((size_t)m->maxN * max_frames);
    std::vector<size_t> o_g(m->scl.size());
    for (size_t j = 0; j < m->scl.size(); ++j) o_g[j] = take(m->scl[j].glob_per_wg * m->scl[j].grid);
    if ((st = hip_check(hipMalloc(&m->mem, off), "polar_mixed_create: hipMalloc")) != POLAR_OK) {
        m->mem = nullptr;
        mixed_release(m);
        return set_error(POLAR_ERR_NO_MEMORY, "polar_mixed_create: device allocation failed");
    }
    char* b = static_cast<char*>(m->mem);
    m->dargs = reinterpret_cast<MixedArgs*>(b + o_args);
    m->dcodes = reinterpret_cast<CodeDev*>(b + o_codes);
    m->gmap = reinterpret_cast<int32_t*>(b + o_gmap);
    m->counts = reinterpret_cast<int32_t*>(b + o_cnt);
    m->lists = reinterpret_cast<int32_t*>(b + o_lists);
    m->queues = reinterpret_cast<int32_t*>(b + o_queues);
    m->ok = reinterpret_cast<uint8_t*>(b + o_ok);
    m->iters = reinterpret_cast<int32_t*>(b + o_it);
    m->scl_ok = reinterpret_cast<uint8_t*>(b + o_sok);
    m->u = reinterpret_cast<uint8_t*>(b + o_u);
    for (size_t j = 0; j < m->scl.size(); ++j) m->glob.push_back(m->scl[j].glob_per_wg ? (void*)(b + o_g[j]) : nullptr);
    std::vector<CodeDev> hc(n_codes);
    for (int c = 0; c < n_codes; ++c) hc[c] = codes[c]->dev();
    st = hip_check(hipMemcpy(m->dcodes, hc.data(), sizeof(CodeDev) * n_codes, hipMemcpyHostToDevice), "copy codes");
    if (st == POLAR_OK)
        st = hip_check(hipMemcpy(m->gmap, gmap.data(), sizeof(int32_t) * n_codes, hipMemcpyHostToDevice), "copy map");
    m->nbr = m->n_groups < kMaxBranches ? m->n_groups : kMaxBranches;
    for (int s = 0; s < m->nbr && st == POLAR_OK; ++s) {
        st = hip_check(hipStreamCreateWithFlags(&m->br[s], hipStreamNonBlocking), "stream create");
        if (st == POLAR_OK) st = hip_check(hipEventCreateWithFlags(&m->ev_join[s], hipEventDisableTiming), "event");
    }
    if (st == POLAR_OK) st = hip_check(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming), "event");
    if (st == POLAR_OK) st = hip_check(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking), "stream create");
    if (st != POLAR_OK) {
        mixed_release(m);
        return st;
    }
    *out = m;
    return ok_status();
}

extern "C" void polar_mixed_free(polar_mixed* m) {
    if (!m) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(m->device);
    hipDeviceSynchronize();
    mixed_release(m);
    hipSetDevice(cur);
}

// everything after the argument block, on `st` (with branches on the plan's streams)
static polar_status mixed_pipeline(polar_mixed* m, hipStream_t st) {
    polar_status r;
    const int nc = m->n_codes, ng = m->n_groups;
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, st, m->counts, 2 * nc);
    const unsigned bgrid = (unsigned)((m->cap + 255) / 256);
    hipLaunchKernelGGL(bucket_kernel, dim3(bgrid), dim3(256), 0, st, m->dargs, nc, m->cap, m->gmap, m->lists,
                       m->counts);
    if ((r = hip_check(hipGetLastError(), "bucket launch")) != POLAR_OK) return r;
    if ((r = hip_check(hipEventRecord(m->ev_fork, st), "event record")) != POLAR_OK) return r;
    for (int s = 0; s < m->nbr; ++s)
        if ((r = hip_check(hipStreamWaitEvent(m->br[s], m->ev_fork, 0), "stream wait")) != POLAR_OK) return r;
    for (int g = 0; g < ng; ++g) {
        hipStream_t bs = m->br[g % m->nbr];
        const polar_code* code = m->codes[m->rep[g]];
        int32_t* queue = m->queues + (int64_t)g * m->cap;
        int32_t* qcount = m->counts + nc + g;
        if ((r = launch_bp_gather(code, &m->dargs->io, m->lists + (int64_t)g * m->cap, m->counts + g, &m->params[g],
                                  m->u, m->maxN, m->iters, m->ok, queue, qcount, m->bp_grid[g], bs)) != POLAR_OK)
            return r;
        if ((r = launch_scl(code, m->scl[g], nullptr, m->L, queue, qcount, 0, m->u, m->scl_ok, nullptr, m->glob[g], bs,
                            &m->dargs->io, m->maxN)) != POLAR_OK)
            return r;
    }
    for (int s = 0; s < m->nbr; ++s) {
        if ((r = hip_check(hipEventRecord(m->ev_join[s], m->br[s]), "event record")) != POLAR_OK) return r;
        if ((r = hip_check(hipStreamWaitEvent(st, m->ev_join[s], 0), "stream wait")) != POLAR_OK) return r;
    }
    hipLaunchKernelGGL(mixed_merge_kernel, dim3((unsigned)m->cap), dim3(64), 0, st, m->dargs, m->dcodes, nc, m->u,
                       (int64_t)m->maxN, m->ok, m->iters, m->scl_ok);
    return hip_check(hipGetLastError(), "mixed merge launch");
}

static polar_status mixed_set_args(polar_mixed* m, int64_t B, const float* llr, const int32_t* code_of_frame,
                                   const int64_t* llr_off, const int64_t* out_off, uint8_t* info_hat,
                                   uint8_t* used_scl, int64_t* stats, hipStream_t stream) {
    if (!m) return set_error(POLAR_ERR_INVALID_ARG, "mixed decode: null plan");
    if (B < 0 || B > m->cap) return set_error(POLAR_ERR_INVALID_ARG, "mixed decode: B outside [0, max_frames]");
    if (B > 0 && (!llr || !code_of_frame || !llr_off || !out_off || !info_hat))
        return set_error(POLAR_ERR_INVALID_ARG, "mixed decode: null buffer");
    int dev = 0;
    polar_status r = hip_check(hipGetDevice(&dev), "get device");
    if (r != POLAR_OK) return r;
    if (dev != m->device) return set_error(POLAR_ERR_INVALID_ARG, "mixed decode: plan belongs to another device");
    MixedArgs a;
    a.io.llr = llr;
    a.io.off = llr_off;
    a.io.code_of = code_of_frame;
    a.io.codes = m->dcodes;
    a.B = B;
    a.code_of_frame = code_of_frame;
    a.out_off = out_off;
    a.info_hat = info_hat;
    a.used_scl = used_scl;
    a.stats = stats;
    hipLaunchKernelGGL(set_args_kernel, dim3(1), dim3(64), 0, stream, m->dargs, a);
    return hip_check(hipGetLastError(), "set args launch");
}

extern "C" polar_status polar_mixed_decode(polar_mixed* m, int64_t B, const float* llr, const int32_t* code_of_frame,
                                           const int64_t* llr_off, const int64_t* out_off, uint8_t* info_hat,
                                           uint8_t* used_scl, int64_t* stats, hipStream_t stream) {
    polar_status r = mixed_set_args(m, B, llr, code_of_frame, llr_off, out_off, info_hat, used_scl, stats, stream);
    if (r != POLAR_OK) return r;
    if (B == 0) return ok_status();
    r = mixed_pipeline(m, stream);
    return r == POLAR_OK ? ok_status() : r;
}

extern "C" polar_status polar_mixed_decode_graph(polar_mixed* m, int64_t B, const float* llr,
                                                 const int32_t* code_of_frame, const int64_t* llr_off,
                                                 const int64_t* out_off, uint8_t* info_hat, uint8_t* used_scl,
                                                 int64_t* stats, hipStream_t stream) {
    polar_status r = mixed_set_args(m, B, llr, code_of_frame, llr_off, out_off, info_hat, used_scl, stats, stream);
    if (r != POLAR_OK) return r;
    if (B == 0) return ok_status();
    if (!m->exec) {
        // capture once on the plan's own stream; the graph reads its inputs
        // through the argument block, so later calls reuse it
        r = hip_check(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
        if (r != POLAR_OK) return r;
        polar_status rp = mixed_pipeline(m, m->cap_stream);
        hipGraph_t g = nullptr;
        r = hip_check(hipStreamEndCapture(m->cap_stream, &g), "end capture");
        if (rp != POLAR_OK) {
            if (g) hipGraphDestroy(g);
            return rp;
        }
        if (r != POLAR_OK) return r;
        hipGraphExec_t ex = nullptr;
        r = hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate");
        if (r != POLAR_OK) {
            hipGraphDestroy(g);
            return r;
        }
        m->graph = g;
        m->exec = ex;
    }
    r = hip_check(hipGraphLaunch(m->exec, stream), "graph launch");
    return r == POLAR_OK ? ok_status() : r;
}
