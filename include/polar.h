/*
 * polar.h -- C ABI of libpolarhip, a hybrid belief-propagation / CRC-aided
 * successive-cancellation-list decoder of polar codes for AMD MI355X (gfx950).
 *
 * Method: Cammerer, Leible, Stahl, Hoydis, ten Brink, "Combining Belief
 * Propagation and Successive Cancellation List Decoding of Polar Codes on a
 * GPU Platform".  Sections cited below are that paper's.
 *
 * Conventions shared by every entry point
 *   - N = 2^n is the block length, x = u G with G = F^{(x)n}, F = [[1,0],[1,1]],
 *     natural index order (Sec. II, Fig. 1).
 *   - A code has K information bits and c CRC bits; the k = K + c
 *     non-frozen positions of u carry the K information bits followed by the
 *     c CRC bits, in ascending index order; frozen positions hold 0.
 *   - Bits are uint8 values 0/1, row-major, one row per frame.
 *   - LLR = ln P(y|0)/P(y|1) (Sec. II-A): a positive LLR favours bit 0.
 *   - "dev" marks a device pointer (e.g. from hipMalloc or a torch tensor),
 *     "host" a host pointer.  The caller owns every batch buffer and every
 *     workspace; the library never allocates during a decode call.
 *   - Every decode/encode call only validates its arguments and enqueues work
 *     on `stream`; results are valid once the stream has been synchronised.
 *     Argument errors are reported synchronously before anything is enqueued.
 *     A device failure is reported as POLAR_ERR_DEVICE by the call that
 *     observes it.  No C++ exception crosses this interface.
 *   - Calls on different streams may run concurrently if they use disjoint
 *     output buffers and workspaces; a polar_code is immutable after
 *     construction and may be shared.
 */
#ifndef POLAR_H
#define POLAR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    POLAR_OK = 0,
    POLAR_ERR_INVALID_ARG = 1, /* a pointer, size or parameter is out of range */
    POLAR_ERR_UNSUPPORTED = 2, /* valid request the library does not implement  */
    POLAR_ERR_NO_MEMORY = 3,   /* host or device allocation failed (construction only) */
    POLAR_ERR_DEVICE = 4,      /* a HIP runtime call failed                       */
    POLAR_ERR_WORKSPACE = 5    /* workspace pointer missing or too small          */
} polar_status;

/* Thread-local, human-readable description of the last error on this thread
 * (empty string after success).  The pointer stays valid until the next call
 * on the same thread. */
const char* polar_last_error(void);

/* ---------------------------------------------------------------------------
 * Code description and construction (Sec. II).
 * The paper decodes a given, arbitrary frozen vector f.  When `frozen` is NULL
 * the library chooses it by the Gaussian approximation of density evolution
 * (Chung, Richardson, Urbanke 2001) at `design_ebn0_db`, with code rate K/N,
 * keeping the k = K + c most reliable positions (ties: the higher index is
 * taken as more reliable).
 * ------------------------------------------------------------------------- */
typedef struct polar_code polar_code;

typedef struct {
    int32_t N;              /* block length: power of two, 8 <= N <= 4096           */
    int32_t K;              /* information bits, excluding the CRC, K >= 1          */
    int32_t crc_bits;       /* c: 0, 8, 16 or 24                                     */
    uint32_t crc_poly;      /* generator without its x^c term; 0 selects the default:
                               0x07 (c=8), 0x1021 (c=16), 0x864CFB (c=24)           */
    double design_ebn0_db;  /* design point of the construction (frozen == NULL)     */
    const uint8_t* frozen;  /* host [N], 1 = frozen, or NULL; must contain exactly
                               N - K - c ones                                        */
    int32_t da_bits;        /* decision-aided list decoding (Sec. II-A): the da_bits
                               most reliable non-frozen positions (Gaussian
                               approximation at design_ebn0_db, ties: higher index)
                               are decided by every path's hard decision without
                               branching; 0 <= da_bits <= K + c, 0 = plain CA-SCL   */
} polar_code_desc;

/* Builds a code and uploads its tables to the current HIP device.  On success
 * *out receives a handle the caller releases with polar_free_code.  Errors:
 * INVALID_ARG (bad sizes, mask with the wrong number of frozen positions),
 * NO_MEMORY, DEVICE. */
polar_status polar_build_code(const polar_code_desc* desc, polar_code** out);

/* Host-only construction of the frozen mask that polar_build_code would use
 * for (N, K, crc_bits, design_ebn0_db) without a given mask: writes N entries
 * (1 = frozen) to host_mask.  Touches no device.  Errors: INVALID_ARG. */
polar_status polar_construct_frozen(int32_t N, int32_t K, int32_t crc_bits, double design_ebn0_db,
                                    uint8_t* host_mask);

/* Releases the host and device tables of a code (NULL is ignored).  The caller
 * must make sure no enqueued work still uses the code. */
void polar_free_code(polar_code* code);

/* Parameters of a built code: any pointer may be NULL. */
polar_status polar_code_params(const polar_code* code, int32_t* N, int32_t* K,
                               int32_t* crc_bits, uint32_t* crc_poly);

/* Copies the frozen mask (1 = frozen) to host memory [N]. */
polar_status polar_code_frozen(const polar_code* code, uint8_t* host_mask);
/* host_mask [N] <- 1 at the decision-aided positions of the list decoder. */
polar_status polar_code_decision_aided(const polar_code* code, uint8_t* host_mask);

/* ---------------------------------------------------------------------------
 * Encoder (Sec. II, Fig. 1).
 * info   dev [B][K]: information bits.
 * u_out  dev [B][N] or NULL: the vector u (info, CRC, zeros on frozen positions).
 * x_out  dev [B][N]: the codeword x = u G.
 * ------------------------------------------------------------------------- */
polar_status polar_encode(const polar_code* code, const uint8_t* info, int64_t B,
                          uint8_t* u_out, uint8_t* x_out, hipStream_t stream);

/* BPSK over AWGN for synthetic workloads: llr = 2 (1 - 2x + sqrt(s2) z) / s2,
 * the LLR of Sec. II-A for a Gaussian channel.
 * x dev [B][N] bits, z dev [B][N] unit-variance noise (the caller draws it),
 * sigma2 dev [B] noise variance per frame, llr dev [B][N] output. */
polar_status polar_channel_awgn(const uint8_t* x, const float* z, const float* sigma2, int64_t B,
                                int32_t N, float* llr, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Belief-propagation decoder (Sec. II-B, Fig. 2).
 * One iteration is a sweep of R messages over stages 2..n+1 followed by a
 * sweep of L messages over stages n..1; inside a stage all N/2 processing
 * elements update at once.  Initialisation L_{i,n+1} = LLR_i,
 * R_{i,1} = llr_max * f_i; outputs LLR(u_i) = L_{i,1} + R_{i,1}.  The rule is
 * min-sum, g(a,b) = sign(a) sign(b) min(|a|,|b|) (rule 0), or the exact
 * ln((1 + e^(a+b)) / (e^a + e^b)) of Sec. II-B (rule 1, single precision,
 * evaluated as sign(a) sign(b) min(|a|,|b|) + ln(1 + e^-|a+b|) -
 * ln(1 + e^-|a-b|)); channel LLRs and every computed message are clipped to
 * +-llr_max.
 * Early stop after each iteration (Sec. II-B): stop = 1 when the re-encoded
 * estimate u_hat G equals the hard decision on LLR(x), stop = 2 when the CRC
 * of u_hat holds, stop = 0 never.
 * ok = CRC holds (stop = 2) or re-encoding check and CRC hold (stop 0, 1;
 * without a CRC only the re-encoding check counts).
 * Weighted (learned) form: when `weights` is given, the g term of every
 * message computed in iteration t, direction d (0 = R, 1 = L), stage column s
 * (0-based, the stage that pairs i with i + 2^s) and output node i is
 * multiplied by weights[((t * 2 + d) * n + s) * N + i] before the addition and
 * the clipping (additions use one fused multiply-add).  weight_layout = 1
 * shares one weight among the nodes of a stage column: weights[(t * 2 + d) * n
 * + s], [weight_iters][2][n] floats.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t max_iter;      /* i_max >= 1 (Sec. III)                               */
    int32_t stop;          /* 0 none, 1 re-encoding check, 2 CRC                  */
    float llr_max;         /* clipping level > 0 (20 in Sec. II-B)                */
    int32_t rule;          /* 0 min-sum, 1 exact (not with weights, not in mixed
                              plans)                                              */
    const float* weights;  /* dev [weight_iters][2][n][N] or NULL                 */
    int32_t weight_iters;  /* >= max_iter when weights != NULL                    */
    int32_t variant;       /* kernel layout: 0 automatic, else a value returned by
                              polar_bp_variants                                   */
    int32_t weight_layout; /* 0 per node [iters][2][n][N], 1 per stage column
                              [iters][2][n]                                       */
} bp_params;

/* llr    dev [B][N] channel LLRs (float32).
 * u_hat  dev [B][N] hard decisions on LLR(u) (frozen positions 0).
 * llr_u  dev [B][N] or NULL: soft output LLR(u) = L_{i,1} + R_{i,1} (Sec. II-B).
 * iters  dev [B] or NULL: iterations run (1..max_iter).
 * ok     dev [B]: verdict as defined above. */
polar_status bp_decode_batch(const polar_code* code, const float* llr, int64_t B,
                             const bp_params* params, uint8_t* u_hat, float* llr_u,
                             int32_t* iters, uint8_t* ok, hipStream_t stream);

/* Kernel layouts of the BP decoder available for a block length: writes up to
 * `cap` variant ids to `ids` and their count to *count.  Used by the autotuner. */
polar_status polar_bp_variants(int32_t N, int32_t* ids, int32_t cap, int32_t* count);

/* ---------------------------------------------------------------------------
 * CRC-aided successive-cancellation list decoder (Sec. II-A), LLR based, min-sum
 * path metrics: a path's metric grows by |LLR(u_i)| whenever its decision
 * differs from the hard decision.  Frozen bits do not branch; at each
 * information bit every path spawns both values and the L candidates of
 * smallest (metric, parent list position, bit) survive, in that order (the
 * "pruned pseudo sort" made a strict total order).  The result is the
 * smallest-metric path whose CRC holds, else the smallest-metric path.
 * L: 1..32, a power of two.
 * frame_ids  dev [B] or NULL: decode frames frame_ids[0..B) of `llr` and write
 *            row frame_ids[q] of the outputs (NULL: frames 0..B-1).
 * u_hat dev rows [N], crc_ok dev [rows], pm dev [rows] or NULL (final metric).
 * ws / ws_bytes: workspace of at least polar_workspace_size(code, B, L, NULL)
 * bytes (may be NULL when that size is 0).
 * ------------------------------------------------------------------------- */
polar_status scl_decode_batch(const polar_code* code, const float* llr, int64_t B, int32_t L,
                              const int32_t* frame_ids, uint8_t* u_hat, uint8_t* crc_ok,
                              float* pm, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Hybrid decoder (Sec. III, Fig. 3): BP with params->max_iter iterations and
 * the params->stop rule on every frame; frames whose verdict is not ok are
 * compacted into a queue on the device (the failed-codeword buffer of Fig. 3) and
 * decoded again from their channel LLRs by the CA-SCL decoder with list size
 * L.  No host round trip: the queue length stays on the device.
 * info_hat  dev [B][K]: information bits of the kept result.
 * used_scl  dev [B] or NULL: 1 when the frame went to the list decoder.
 * stats     dev int64 [8] or NULL, accumulated (not cleared):
 *           [0] frames, [1] BP ok, [2] SCL frames, [3] BP iterations summed,
 *           [4] SCL frames whose CRC failed, [5..7] reserved (0).
 * Graphs: the kernels of a call are fixed by (device, code, B, params, L,
 * the buffer pointers, the list decoder's tuning settings).  The first call
 * with such a combination launches them directly; the second captures them
 * into one hipGraph and every later call with the same combination replays
 * it on `stream` (the kernels read the buffers, including the weights, when
 * they run, so their contents may change between calls).  The library keeps
 * the graphs of the 8 most recently used combinations.  Calls on a stream
 * that is being captured launch directly.  polar_set_hybrid_graphs(0) turns
 * the replay off (process-wide), 1 (the default) on.
 * ------------------------------------------------------------------------- */
polar_status hybrid_decode_batch(const polar_code* code, const float* llr, int64_t B,
                                 const bp_params* params, int32_t L, uint8_t* info_hat,
                                 uint8_t* used_scl, int64_t* stats, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

polar_status polar_set_hybrid_graphs(int32_t mode);
int32_t polar_get_hybrid_graphs(void);

/* ---------------------------------------------------------------------------
 * hybrid_decode_batch for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same decode, arguments and results, without a workspace
 * argument.  The workspace lives in a fixed 64 MiB array of device memory
 * that the library holds on each device it runs on until the process ends;
 * the call allocates nothing.  The batch state takes about B * (N + 10)
 * bytes (plus alignment) and the list decoder's global slice at least one
 * workgroup's share (L * N * 4 + k * L bytes when its state does not fit in
 * LDS); a batch that does not fit returns POLAR_ERR_INVALID_ARG before
 * anything is enqueued.  At N = 1024, L = 32 up to about 64000 frames fit.
 * With less room than hybrid_decode_batch would take, the list decoder runs
 * fewer persistent workgroups (same results, lower throughput when many
 * frames fail BP).  All calls on one device share that array: calls that can
 * overlap on a device (other streams, other threads) race and must be
 * serialised by the caller; a call does not depend on what an earlier one
 * left there.
 * ------------------------------------------------------------------------- */
polar_status hybrid_decode_batch_static(const polar_code* code, const float* llr, int64_t B,
                                        const bp_params* params, int32_t L, uint8_t* info_hat,
                                        uint8_t* used_scl, int64_t* stats, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Pipelined hybrid over a sequence of batches: the asynchronous BP / SCL
 * scheduling of Sec. III (Fig. 3) on two streams.  For batch j, BP and the
 * compaction of its failed frames run on stream_bp; its CA-SCL and the merge
 * run on stream_scl once they are done, so the list decoding of batch j
 * overlaps the BP of the following batches.  The workspace holds two
 * per-batch states (batch j + 2 waits for the merge of batch j); the list
 * decoder's global slice is shared, since list decodes follow one another on
 * stream_scl.
 * llr, info_hat, used_scl: host arrays of nbatch device pointers ([B][N],
 * [B][K], [B]; used_scl may be NULL or hold NULL entries); batches may share
 * an input buffer, not an output buffer (the BP of batch j + 1 writes its
 * kept frames' information bits while batch j's list-decoded ones are merged).  Results and stats (accumulated as in hybrid_decode_batch)
 * are complete when work enqueued on stream_bp after the call completes:
 * stream_bp finally waits for stream_scl.  The two streams must differ.
 * ws: at least polar_pipeline_workspace_size(code, B, L, params) bytes.
 * ------------------------------------------------------------------------- */
polar_status hybrid_decode_pipelined(const polar_code* code, int64_t nbatch, const float* const* llr, int64_t B,
                                     const bp_params* params, int32_t L, uint8_t* const* info_hat,
                                     uint8_t* const* used_scl, int64_t* stats, void* ws, size_t ws_bytes,
                                     hipStream_t stream_bp, hipStream_t stream_scl);
polar_status polar_pipeline_workspace_size(const polar_code* code, int64_t B, int32_t L, const bp_params* params,
                                           size_t* bytes);
/* Workgroups per CU the pipelined hybrid's BP may occupy at a time (1..64),
 * or 0 (the default) for no limit.  With a limit, BP runs as a persistent grid
 * of that many workgroups per CU (min-sum rule, no weights or one weight per
 * stage column; other parameters ignore the limit), which leaves registers and
 * LDS for the list decoder of the previous batch to run beside it.
 * Process-wide; host only. */
polar_status polar_set_pipeline_bp_occupancy(int32_t wgs_per_cu);
int32_t polar_get_pipeline_bp_occupancy(void);
/* Workgroups per CU the pipelined hybrid's list decoder may run (1..64), or 0
 * (the default) for as many as its registers and LDS allow on a CU.  The
 * persistent list-decoder workgroups then walk the queue of failed frames in
 * fewer, longer runs beside the next batch's BP; results are the same for every
 * setting.  Only hybrid_decode_pipelined reads it.  Process-wide; host only. */
polar_status polar_set_pipeline_scl_occupancy(int32_t wgs_per_cu);
int32_t polar_get_pipeline_scl_occupancy(void);

/* ---------------------------------------------------------------------------
 * Ragged batches that mix several codes (block lengths and rates): the
 * hybrid decoder of Sec. III applied frame by frame with each frame's code.
 * A plan holds up to 16 codes (all of the current device), the BP parameters
 * (unweighted; params->variant is replaced by variants[c] when variants is
 * not NULL, 0 = default layout; codes of one block length share the BP
 * kernel of the first of them, and so its layout), the list size and its own
 * device workspace
 * for up to max_frames frames per call; creating it allocates, calls do not.
 * A call decodes B frames in any order: frame f uses code code_of_frame[f]
 * (frames with an id outside [0, n_codes) are skipped), its N LLRs start at
 * element llr_off[f] of llr and its K information bits are written from
 * element out_off[f] of info_hat (all dev; the caller keeps the offsets inside
 * its buffers).  used_scl dev [B] or NULL; stats as in hybrid_decode_batch.
 * On the device the frames are bucketed by block length (codes shorter than
 * 32 bits: by code); each bucket's BP is a persistent kernel that decodes
 * every frame with its own code and appends the failed frames to a queue
 * drained by one persistent CA-SCL kernel, again per frame's code; the
 * buckets' chains are concurrent branches on the plan's streams; a merge
 * writes the results.
 * polar_mixed_decode enqueues the kernels; polar_mixed_decode_graph replays
 * the same work as one hipGraph, captured on its first call on the plan
 * (the kernels read the per-call buffers through a device argument block
 * that a one-thread kernel fills before the graph runs).  Results are
 * complete when later work on `stream` runs.  One call at a time per plan.
 * ------------------------------------------------------------------------- */
typedef struct polar_mixed polar_mixed;
polar_status polar_mixed_create(const polar_code* const* codes, int32_t n_codes, int64_t max_frames,
                                const bp_params* params, int32_t L, const int32_t* variants, polar_mixed** out);
polar_status polar_mixed_decode(polar_mixed* m, int64_t B, const float* llr, const int32_t* code_of_frame,
                                const int64_t* llr_off, const int64_t* out_off, uint8_t* info_hat,
                                uint8_t* used_scl, int64_t* stats, hipStream_t stream);
polar_status polar_mixed_decode_graph(polar_mixed* m, int64_t B, const float* llr, const int32_t* code_of_frame,
                                      const int64_t* llr_off, const int64_t* out_off, uint8_t* info_hat,
                                      uint8_t* used_scl, int64_t* stats, hipStream_t stream);
void polar_mixed_free(polar_mixed* m);

/* Workspace bytes needed by scl_decode_batch (params == NULL) or
 * hybrid_decode_batch (params != NULL) for B frames and list size L. */
polar_status polar_workspace_size(const polar_code* code, int64_t B, int32_t L,
                                  const bp_params* params, size_t* bytes);

/* Per-workgroup LDS budget of the list decoder in bytes, 4096..163840, or 0
 * (the default: a CU's 160 KB divided by the number of the kernel's one-wave
 * workgroups its registers let share a CU).  A list decode keeps as much of
 * its state in LDS as the budget allows: when it does not all fit, the per-bit
 * trace moves to the workspace's global slice first, then the largest LLR
 * tree levels do.  A smaller budget lets more workgroups share a CU.
 * Process-wide; it applies to plans made afterwards, so query workspace sizes
 * again after a change.  POLAR_ERR_INVALID_ARG outside the range.  Host only;
 * polar_get_scl_lds_budget returns the setting (0 = automatic). */
polar_status polar_set_scl_lds_budget(int64_t bytes);
int64_t polar_get_scl_lds_budget(void);

/* How the list decoder finds the L survivors among the 2L candidates of a
 * branching bit (Sec. II-A describes the first two): 1 the pruned pseudo sort
 * -- each candidate counts the candidates before it; 2 the bitonic sorting
 * network across the wavefront, run until the L smallest candidates are
 * separated (list sizes 8 and 32, N >= 32); 3 threshold
 * selection -- the L-th smallest metric found bit by bit with wavefront
 * ballots (list sizes 8, 16 and 32, N >= 32); other lists use the pseudo
 * sort.  0 (default) automatic: the bitonic network for L = 8 and 32, where
 * it measured fastest on MI355X, the pseudo sort otherwise.  All decide
 * survival by the strict order (metric, parent position, bit) and keep the
 * survivors in the order the candidates are listed (parent position, then
 * bit), so results are identical.  Process-wide; host only; mode outside 0..3
 * gives POLAR_ERR_INVALID_ARG. */
polar_status polar_set_scl_ranking(int32_t mode);
int32_t polar_get_scl_ranking(void);

/* ---------------------------------------------------------------------------
 * Weighted (learned) min-sum BP -- not in the paper; trains the weights of the
 * weighted form of bp_decode_batch.  W: dev float [T][2][n][N] as in bp_params.
 * ------------------------------------------------------------------------- */

/* T weighted iterations, no early stop.  llr_u dev [B][N] (soft output
 * LLR(u) = L_{i,1} + R_{i,1}), u_hat dev [B][N] (hard decisions), saved dev
 * [B][T][2][n][N] or NULL: every message produced, saved[f][t][d][s][i] = the
 * row of direction d (0 = R, row s+1; 1 = L, row s) that column s produced in
 * iteration t -- the input of wbp_backward. */
polar_status wbp_forward(const polar_code* code, const float* llr, int64_t B, const float* W, int32_t T,
                         float llr_max, int32_t variant, float* llr_u, uint8_t* u_hat, float* saved,
                         hipStream_t stream);

/* Binary cross-entropy of P(u_i = 1) = sigmoid(-llr_u_i) against u_true (dev
 * [B][N] bits) over the non-frozen positions: loss dev [B] or NULL (per frame,
 * times scale), dlam dev [B][N] = scale * d(loss)/d(llr_u) (0 on frozen
 * positions).  Computed in double precision, stored as float. */
polar_status wbp_bce(const polar_code* code, const float* llr_u, const uint8_t* u_true, int64_t B, double scale,
                     float* loss, float* dlam, hipStream_t stream);

/* The same loss after every one of the T iterations (a loss per iteration,
 * summed): LLR(u) after iteration t is read from saved (wbp_forward's saved
 * rows: L row 0 of iteration t plus the frozen prior).  loss dev [B] or NULL,
 * dlam dev [B][T][N] = scale * d(loss)/d(LLR(u) after iteration t).  Must run
 * before wbp_backward, which overwrites `saved`. */
polar_status wbp_bce_multi(const polar_code* code, const float* saved, const uint8_t* u_true, int64_t B, int32_t T,
                           double scale, float* loss, float* dlam, hipStream_t stream);

/* Frame-failure surrogate after every one of the T iterations: with S_t the
 * binary cross-entropy above summed over the non-frozen positions of LLR(u)
 * after iteration t (read from wbp_forward's saved rows, as wbp_bce_multi
 * does), and the bits taken as independent, e^{-S_t} is the probability that
 * all decisions after iteration t are right; the frame's loss is
 * prod_t (1 - e^{-S_t}), the probability that no iteration gets the whole
 * frame right -- a smooth stand-in for a BP failure within T iterations, the
 * frames the hybrid of Sec. III hands to the list decoder.  loss dev [B] or
 * NULL (times scale), dlam dev [B][T][N] = scale * d(loss)/d(LLR(u) after
 * iteration t).  1 <= T <= 256.  Double precision inside, float stored.  Must
 * run before wbp_backward, which overwrites `saved`. */
polar_status wbp_frame_loss(const polar_code* code, const float* saved, const uint8_t* u_true, int64_t B,
                            int32_t T, double scale, float* loss, float* dlam, hipStream_t stream);

/* Expected-iterations loss of an early-stopping decoder: with q_t = 1 -
 * e^{-S_t} as above and P_u = prod_{t<=u} q_t the probability (bits taken as
 * independent) that the frame is still undecided after iteration u, the
 * frame's loss is sum_{u<T} P_u + fail_weight * P_T: the expected number of
 * iterations beyond the first that a decoder stopping at the first right
 * iteration runs, plus fail_weight per frame still undecided after T (the
 * hybrid of Sec. III then runs the list decoder, which costs about as much as
 * fail_weight iterations).  Same arguments as wbp_frame_loss; fail_weight >= 0
 * (POLAR_ERR_INVALID_ARG otherwise). */
polar_status wbp_iteration_loss(const polar_code* code, const float* saved, const uint8_t* u_true, int64_t B,
                                int32_t T, double fail_weight, double scale, float* loss, float* dlam,
                                hipStream_t stream);

/* One weight per stage column (the column layout of bp_params): W dev
 * [T][2][n][N] = Wc dev [T][2][n] repeated over the N nodes of each column
 * (wbp_column_weights); dWc dev [T][2][n] = dW dev [T][2][n][N] summed over
 * each column's nodes in node order, in double (wbp_column_grad) -- the
 * gradient of a weight the whole column shares. */
polar_status wbp_column_weights(const polar_code* code, const float* Wc, int32_t T, float* W, hipStream_t stream);
polar_status wbp_column_grad(const polar_code* code, const float* dW, int32_t T, float* dWc, hipStream_t stream);

/* Reverse-mode gradient of the weighted BP: dW dev [T][2][n][N] = sum over the
 * B frames (in frame order, accumulated in double) of d(loss)/dW given dlam
 * dev [B][dlam_iters][N]: d(loss)/d(llr_u) after the last iteration
 * (dlam_iters = 1) or after every iteration (dlam_iters = T); dllr dev [B][N]
 * or NULL = d(loss)/d(llr).  `saved` (from wbp_forward with the same llr, W,
 * T) is used as scratch and is undefined afterwards.  Deterministic. */
polar_status wbp_backward(const polar_code* code, const float* llr, int64_t B, const float* W, int32_t T,
                          float llr_max, int32_t variant, float* saved, const float* dlam, int32_t dlam_iters,
                          float* dW, float* dllr, hipStream_t stream);

/* One Adam step (Kingma and Ba, 2015) on `count` float parameters, step >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr m_hat / (sqrt(v_hat) + eps)
 * with bias corrections 1 - b^step.  All arrays dev, updated in place. */
polar_status polar_adam_step(float* w, const float* g, float* m, float* v, int64_t count, int32_t step, float lr,
                             float beta1, float beta2, float eps, hipStream_t stream);

/* The same step followed by a projection of each weight onto [lo, hi]
 * (POLAR_ERR_INVALID_ARG unless lo <= hi).  The learned hybrid keeps its
 * weights within [0, 1]: the decoder then never amplifies a check-node
 * message and bp_decode_batch skips a clip that cannot act. */
polar_status polar_adam_step_bounded(float* w, const float* g, float* m, float* v, int64_t count, int32_t step,
                                     float lr, float beta1, float beta2, float eps, float lo, float hi,
                                     hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* POLAR_H */
