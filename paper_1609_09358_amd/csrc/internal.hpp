// internal.hpp -- definitions shared by the host side and the kernels of
// libpolarhip (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hsa/hsa.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/polar.h"

namespace polarhip {

// Work-item and workgroup indices read from the registers the dispatch
// initialises, grid and workgroup sizes from the dispatch packet.  HIP's
// index variables go through device-library functions built with packed FP32
// on; the inliner keeps them out of code built with it off, so every read
// would be a call and the workgroup id a per-lane value.
__device__ __forceinline__ int lid_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int64_t gid_x() { return (int64_t)__builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ const hsa_kernel_dispatch_packet_t* dispatch_packet() {
    return (const hsa_kernel_dispatch_packet_t*)__builtin_amdgcn_dispatch_ptr();
}
__device__ __forceinline__ int wg_size_x() { return (int)dispatch_packet()->workgroup_size_x; }
__device__ __forceinline__ int64_t num_groups_x() {
    const hsa_kernel_dispatch_packet_t* p = dispatch_packet();
    const int64_t wg = p->workgroup_size_x;
    return ((int64_t)p->grid_size_x + wg - 1) / wg;
}

// Device-side view of a code, passed to kernels by value.
struct CodeDev {
    const uint32_t* frozen_bits;  // [max(N/32,1)] bit i of word i/32 set = frozen
    const int16_t* info_pos;      // [k] non-frozen positions in ascending order
    const uint32_t* syn;          // [N] CRC syndrome contribution of u_i = 1
    const uint32_t* syn_nib;      // [N/4][16] syndrome of each nibble value
    const uint32_t* enc_crc;      // [K] CRC of the unit vector at info bit q
    const uint32_t* da_bits;      // [max(N/32,1)] decision-aided positions of the list decoder
    int32_t N, n, K, c, k;
};

}  // namespace polarhip

struct polar_code {
    int32_t N, n, K, c, k;
    uint32_t poly;
    int device;
    uint64_t serial;                // distinct for every code built in the process
    std::vector<uint8_t> frozen;    // host [N]
    std::vector<int16_t> info_pos;  // host [k]
    std::vector<uint8_t> da;        // host [N], decision-aided positions
    // device allocations (owned)
    uint32_t* d_frozen_bits = nullptr;
    int16_t* d_info_pos = nullptr;
    uint32_t* d_syn = nullptr;
    uint32_t* d_syn_nib = nullptr;
    uint32_t* d_enc_crc = nullptr;
    uint32_t* d_da_bits = nullptr;
    polarhip::CodeDev dev() const {
        polarhip::CodeDev d;
        d.frozen_bits = d_frozen_bits;
        d.info_pos = d_info_pos;
        d.syn = d_syn;
        d.syn_nib = d_syn_nib;
        d.enc_crc = d_enc_crc;
        d.da_bits = d_da_bits;
        d.N = N;
        d.n = n;
        d.K = K;
        d.c = c;
        d.k = k;
        return d;
    }
};

namespace polarhip {

// error reporting (thread local)
polar_status set_error(polar_status st, const std::string& msg);
polar_status ok_status();
polar_status hip_check(hipError_t e, const char* what);

// launch helpers implemented in the kernel translation units
// wgs_per_cu > 0: at most that many BP workgroups per CU at a time (a
// persistent grid), where such a kernel exists (min-sum, unweighted or
// per-stage weights); otherwise one workgroup per frame group
// info_out (or null): [B][K] information bits of the frames whose verdict is ok
polar_status launch_bp(const polar_code* code, const float* llr, int64_t B, const bp_params* p,
                       uint8_t* u_hat, float* llr_u, int32_t* iters, uint8_t* ok,
                       hipStream_t stream, int wgs_per_cu = 0, uint8_t* info_out = nullptr);
polar_status launch_bp_save(const polar_code* code, const float* llr, int64_t B, int T, float llr_max,
                            const float* W, int variant, uint8_t* u_hat, float* llr_u, uint8_t* ok, float* saved,
                            hipStream_t stream);
// Per-call inputs of a ragged batch, read by the kernels from device memory
// (so a captured graph stays valid across calls with other buffers)
struct MixedIo {
    const float* llr;     // LLR rows
    const int64_t* off;   // row of frame f starts at element off[f]
    // several codes in one launch (or null): frame f is decoded with
    // codes[code_of[f]] instead of the kernel's code argument
    const int32_t* code_of;
    const CodeDev* codes;
};

// persistent BP over a device list of frame ids with ragged row offsets;
// failed frames are appended to fail_ids
polar_status bp_gather_grid(const polar_code* code, const bp_params* p, int64_t max_frames, int* grid);
// u_hat row of frame f: f * u_stride
polar_status launch_bp_gather(const polar_code* code, const MixedIo* io, const int32_t* ids, const int32_t* count,
                              const bp_params* p, uint8_t* u_hat, int64_t u_stride, int32_t* iters, uint8_t* ok,
                              int32_t* fail_ids, int32_t* fail_count, int grid, hipStream_t stream);
bool bp_variant_supported(int n, int variant);
int bp_default_variant(int n);
int bp_list_variants(int n, int32_t* ids, int cap);

struct SclPlan {
    int gl;              // LLR levels >= gl live in the global slice
    size_t lds_bytes;    // dynamic LDS per workgroup
    int trace_glob;      // 1: the per-block trace lives in the global slice
    int tb_off;          // LDS byte offset of the trace when !trace_glob
    size_t trace_off;    // byte offset of the trace inside the global slice
    size_t glob_per_wg;  // global slice bytes per workgroup (levels >= gl, trace)
    int grid;            // workgroups launched
    int lay_n;           // log2 of the largest block length the layout holds
};
polar_status scl_plan(const polar_code* code, int L, int64_t max_frames, SclPlan* plan);
// a plan that holds any code with n <= max_n (n >= 5)
polar_status scl_plan_dims(int max_n, int L, int64_t max_frames, SclPlan* plan);
// io (optional): LLR rows of a ragged batch (frame f at element io->off[f]),
// u_hat rows then at f * u_stride
polar_status launch_scl(const polar_code* code, const SclPlan& plan, const float* llr, int L,
                        const int32_t* frame_ids, const int32_t* count_dev, int64_t count_host,
                        uint8_t* u_hat, uint8_t* crc_ok, float* pm, void* glob,
                        hipStream_t stream, const MixedIo* io = nullptr, int64_t u_stride = 0);

int device_cu_count();

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace polarhip
