// sre2_ctx.h - the library context (workspace owned per device and stream)
// and the internal entry points the serving loop builds on.  Not public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "sre2_internal.h"

namespace sre2 {
// Default upper bound of the two-pass slab of a context (sre2_set_scratch_limit).
constexpr size_t kDefaultScratchLimit = size_t(32) << 30;
}  // namespace sre2

struct sre2_ctx {
    int device = 0;
    size_t scratch_limit = sre2::kDefaultScratchLimit;  // halved on allocation failure, per call
    bool row_pairs = true;  // row-pair half slabs for the M2 forms (sre2_set_row_pairs)
    void* psi_work = nullptr;
    size_t psi_work_bytes = 0;
    double* sx = nullptr;  // S_x when the caller passes no partials buffer
    size_t sx_bytes = 0;
    void* scratch = nullptr;  // two-pass slab
    size_t scratch_bytes = 0;
    double* part = nullptr;  // two-pass column-group partials of one chunk
    size_t part_bytes = 0;
    double* red = nullptr;  // norm partials, flags, S partials
    size_t red_bytes = 0;
    double* pack_ws = nullptr;  // packed launches: per-state workspace blocks
    size_t pack_ws_bytes = 0;
    void* pack_work = nullptr;  // packed launches: converted inputs
    size_t pack_work_bytes = 0;
    // optional per-launch timing (sre2_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> events;       // pool, reused between reads
    std::vector<int> pending;             // kind of each recorded (start, stop) pair
};

namespace sre2 {
// Device buffers of one evaluation.  The context path grows them with
// hipMalloc; the allocation-free entry point carves them out of a fixed
// device array.  Nothing in them needs to start at zero: every kernel writes
// each entry it later reads.
struct Workspace {
    void* psi_work = nullptr;  // input in the form's precision (when the dtype differs)
    double* red = nullptr;     // norm partials, flags, S partials, scale, n (red_doubles())
    double* sx = nullptr;      // S_x of every shift (when the caller passes none)
    void* scratch = nullptr;   // two-pass slab
    double* part = nullptr;    // two-pass column-group partials of one chunk
    size_t limit = 0;          // slab bytes available: sets the chunk size
    bool pairs = true;         // the plain and split M2 forms take row-pair slabs above 2^L
};
constexpr size_t red_doubles() { return 3 * (size_t)kMaxRed + 2; }

// sre2_m2 on the buffers of ws (no allocation, no timing).
int ws_m2(const Workspace& ws, const void* psi, int N, int dtype, int form, hipStream_t st,
          double* out, double* partials);
// Byte offsets of the parts of a Workspace inside one buffer of `bytes`
// (reduction buffer at 0, every part 256-byte aligned) and the slab bytes
// (limit) for a call of this shape; SRE2_ESCRATCH when even one shift per
// chunk does not fit.
int ws_layout(int N, int dtype, int form, bool need_sx, size_t bytes, size_t* psi_work_off,
              size_t* sx_off, size_t* part_off, size_t* slab_off, size_t* limit);
// Host-side argument check of (N, dtype, form), as sre2_m2 does it.
int ctx_validate_form(int N, int dtype, int form);

// One full evaluation of one state (sre2_m2 without partials).
int ctx_m2_one(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, hipStream_t st,
               double* out);
// Up to kMaxPack states of one N <= ctx_fused_max(form) in packed launches.
int ctx_m2_pack(sre2_ctx* ctx, const void* const* psi, int count, int N, int dtype, int form,
                double* const* outs, hipStream_t st);
int ctx_fused_max(int form);
// Grow the packed-launch workspace for every N up to `N` (so that it never
// has to be reallocated while packed work is in flight).
int ctx_reserve_pack(sre2_ctx* ctx, int N, int form);
}  // namespace sre2
