// sre2_api.hip - C ABI of libsre2 (declared in include/sre2.h): argument
// validation, workspace management and the launch sequence of one M2
// evaluation.  All arithmetic runs in the kernels of sre2_kernels.hip.
//
// Launch sequence of sre2_m2 on the caller's stream:
//   [k_convert]        input -> working precision copy (only if dtype != form's)
//   k_norm_part        FP64 partial norms + non-finite flags
//   shift sums         k_tiny | k_fused | per chunk: k_pass1, k_pass2, k_group_sum
//   k_sum_part         fixed-range FP64 partial sums of S_x
//   k_final            S, n, M2 = -log2(S / (2^N n^4)), status
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <new>
#include <vector>

#include "../../include/sre2.h"
#include "sre2_internal.h"
#include "sre2_ctx.h"

using namespace sre2;



namespace {


struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Fault injection for tests of the error paths, from the host only (no
// kernel is made to fail): SRE2_FAULT=alloc (every workspace allocation
// fails), alloc_4g (allocations above 4 GiB fail), launch (the transform
// launches of an evaluation report a launch error after the staging and norm
// kernels were enqueued).
int fault_injected(const char* what) {
    const char* f = getenv("SRE2_FAULT");
    return f && strcmp(f, what) == 0;
}

int ensure(void** buf, size_t* have, size_t need) {
    if (*have >= need && *buf) return SRE2_OK;
    if (fault_injected("alloc")) return SRE2_ENOMEM;
    // a device with little free memory: requests above 4 GiB fail
    if (need > (size_t(4) << 30) && fault_injected("alloc_4g")) return SRE2_ENOMEM;
    if (*buf) {
        if (hipFree(*buf) != hipSuccess) return SRE2_EHIP;
        *buf = nullptr;
        *have = 0;
    }
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, need);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return SRE2_ENOMEM;
    }
    if (e != hipSuccess) return SRE2_EHIP;
    *buf = p;
    *have = need;
    return SRE2_OK;
}

bool form_ok(int form) {
    return form == SRE2_FORM_FP32 || form == SRE2_FORM_FP64 || form == SRE2_FORM_FP32_HERM ||
           form == SRE2_FORM_FP64_HERM || form == SRE2_FORM_SPLIT_F16 ||
           form == SRE2_FORM_SPLIT_BF16;
}
// Split kind of the kernels: 0 none, 1 FP16 halves, 2 BF16 halves.
int split_kind(int form) {
    return form == SRE2_FORM_SPLIT_F16 ? 1 : form == SRE2_FORM_SPLIT_BF16 ? 2 : 0;
}
bool is_split(int form) { return split_kind(form) != 0; }
bool is_f64(int form) { return form == SRE2_FORM_FP64 || form == SRE2_FORM_FP64_HERM; }
bool is_herm(int form) { return form == SRE2_FORM_FP32_HERM || form == SRE2_FORM_FP64_HERM; }
bool dtype_ok(int dtype) { return dtype == SRE2_C64 || dtype == SRE2_C128; }

int elem_bytes(int dtype) { return dtype == SRE2_C64 ? 8 : 16; }
int work_dtype(int form) { return is_f64(form) ? kC128 : kC64; }

int fused_max(int form) { return is_f64(form) ? fused_max_n<double>() : fused_max_n<float>(); }
// pass-1 row bits of a slab of NS bits
int row_bits(int form, int NS) {
    return is_f64(form) ? pass1_row_bits<double>(NS) : pass1_row_bits<float>(NS);
}
int herm_min(int form) { return is_f64(form) ? herm_min_n<double>() : herm_min_n<float>(); }
int64_t col_tiles(int N, int form, bool herm) {
    return is_f64(form) ? pass2_col_tiles<double>(N, herm) : pass2_col_tiles<float>(N, herm);
}

// Two-pass chunking: shifts per chunk (power of two) and column groups per shift.
struct Chunking {
    int64_t cs = 0;
    int P = 1;
};

// Slab bits of one shift and pass-1 row bits of a slab kind (kSlabFull,
// kSlabHerm, kSlabPairs).
int slab_bits(int N, int slab) { return N - (slab == kSlabFull ? 0 : 1); }
int slab_rows(int form, int N, int slab) {
    return row_bits(form, slab == kSlabHerm ? N - 1 : N);
}

Chunking chunking(int N, int form, int slab, int64_t x_count, size_t limit) {
    Chunking c;
    if (N <= fused_max(form)) return c;
    const int L = slab_rows(form, N, slab);
    const size_t bytes = (size_t(1) << slab_bits(N, slab)) * (size_t)elem_bytes(work_dtype(form));
    int64_t cs = 1;
    while ((size_t)(cs * 2) * bytes <= limit && cs * 2 <= x_count && cs * 2 <= (int64_t(1) << L))
        cs *= 2;
    c.cs = cs;
    // Column groups per shift depend on (N, form) only - never on the chunk
    // size - so the order of the FP64 partial sums, and hence every result
    // bit, is independent of the scratch limit.  The row pairs keep the
    // full slab's pass-2 tiles.  At most 16 groups: each workgroup then loops
    // over several column tiles and loads the next during each transform
    // (N = 20: 3 % faster than 64 groups, 1-2 % than 32).
    const int64_t tiles = col_tiles(N, form, slab == kSlabHerm);
    int P = 1;
    while (P < 16 && P * 2 <= tiles) P *= 2;
    c.P = P;
    return c;
}

// The shifts [x0, x0 + xc) of a two-pass evaluation split into at most two
// ranges by slab kind: the full slab below 2^L, the half slab (Hermitian
// pair; row pairs of the plain and split M2 forms when `pairs`) above.
struct SlabRange {
    int slab;
    int64_t x0, xc;
};
int slab_ranges(int N, int form, bool pairs, int64_t x0, int64_t xc, SlabRange* out) {
    const int64_t x1 = x0 + xc;
    int half = kSlabFull;
    if (is_herm(form))
        half = kSlabHerm;
    else if (pairs)
        half = kSlabPairs;
    int64_t split = x1;
    if (half != kSlabFull) {
        const int64_t lim =
            half == kSlabHerm ? int64_t(1) << slab_rows(form, N, half)
            : is_f64(form)    ? pair_first_shift<double>(N, 0)
                              : pair_first_shift<float>(N, split_kind(form));
        split = x0 > lim ? x0 : (x1 < lim ? x1 : lim);
    }
    int k = 0;
    if (split > x0) out[k++] = SlabRange{kSlabFull, x0, split - x0};
    if (x1 > split) out[k++] = SlabRange{half, split, x1 - split};
    return k;
}

// Reduction blocks of a state of n amplitudes / shifts: about 1024 values per
// block (four per thread), so that small states do not wait on one block's
// long dependent chain; fixed by n, hence part of every result's fixed order.
int red_blocks(int64_t n) {
    int64_t b = n >> 10;
    if (b < 1) b = 1;
    if (b > kMaxRed) b = kMaxRed;
    return (int)b;
}

// Bracket one launch with a pair of pooled events when timing is enabled.
struct Timed {
    sre2_ctx* ctx;
    hipStream_t st;
    int kind;
    size_t slot = 0;
    bool on = false;
    Timed(sre2_ctx* c, hipStream_t s, int k) : ctx(c), st(s), kind(k) {
        if (!ctx || !ctx->timing) return;
        slot = ctx->pending.size() * 2;
        while (ctx->events.size() < slot + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ctx->events.push_back(e);
        }
        on = hipEventRecord(ctx->events[slot], st) == hipSuccess;
    }
    ~Timed() {
        if (on && hipEventRecord(ctx->events[slot + 1], st) == hipSuccess)
            ctx->pending.push_back(kind);
    }
};

int hip_status(hipError_t e) { return e == hipSuccess ? SRE2_OK : SRE2_EHIP; }

int validate(const sre2_ctx* ctx, const void* psi, int N, int dtype, int form) {
    if (!ctx || !psi) return SRE2_EINVAL;
    if (N < 1 || N > SRE2_MAX_N) return SRE2_EINVAL;
    if (!dtype_ok(dtype)) return SRE2_EDTYPE;
    if (!form_ok(form)) return SRE2_EFORM;
    if (N > (is_f64(form) ? max_n<double>() : max_n<float>())) return SRE2_EFORM;
    return SRE2_OK;
}

// Layout of Workspace::red: norm partials, non-finite flags, S partials
// (kMaxRed doubles each), one int (the split form's scale exponent) in a
// double, then n (the histogram's normalisation).
struct Red {
    double* npart;
    double* nflag;
    double* spart;
    int* se;
    double* nrm;
};

Red red_of(double* red) {
    Red r;
    r.npart = red;
    r.nflag = red + kMaxRed;
    r.spart = red + 2 * kMaxRed;
    r.se = reinterpret_cast<int*>(red + 3 * kMaxRed);
    r.nrm = red + 3 * kMaxRed + 1;
    return r;
}

// Stage the input in the form's working precision (into ws.psi_work when
// the dtype differs); returns the pointer the kernels read.
int stage_input(sre2_ctx* tctx, const Workspace& ws, const void* psi, int N, int dtype, int form,
                hipStream_t st, const void** work) {
    const int wd = work_dtype(form);
    if (wd == dtype) {
        *work = psi;
        return SRE2_OK;
    }
    Timed tm(tctx, st, SRE2_KIND_AUX);
    *work = ws.psi_work;
    return hip_status(launch_convert(psi, dtype, ws.psi_work, wd, int64_t(1) << N, st));
}

// Two-pass over [x0, x0 + xc) with one slab kind, chunks sized by ws.limit.
int two_pass(sre2_ctx* tctx, const Workspace& ws, const void* work, int N, int form, int slab,
             int64_t x0, int64_t xc, double* Sx, const int* se, const Spec* spec,
             hipStream_t st) {
    const bool f64 = is_f64(form);
    const int split = split_kind(form);
    const Chunking ch = chunking(N, form, slab, xc, ws.limit);
    // row pairs: a chunk stays inside one block of 2^L shifts (one row part
    // x >> L per launch, so every workgroup takes the same specialisation)
    const int64_t blk = slab == kSlabPairs ? int64_t(1) << slab_rows(form, N, slab) : 0;
    for (int64_t c0 = 0, cs = 0; c0 < xc; c0 += cs) {
        // a short last chunk keeps the same column grouping
        cs = xc - c0 < ch.cs ? xc - c0 : ch.cs;
        if (blk) {
            const int64_t to_edge = blk - ((x0 + c0) & (blk - 1));
            cs = cs < to_edge ? cs : to_edge;
        }
        hipError_t e;
        {
            Timed tm(tctx, st, SRE2_KIND_PASS1);
            e = f64 ? launch_pass1<double>(work, N, slab, split, x0 + c0, (int)cs, ws.scratch, se,
                                           st)
                    : launch_pass1<float>(work, N, slab, split, x0 + c0, (int)cs, ws.scratch, se,
                                          st);
        }
        if (e != hipSuccess) return SRE2_EHIP;
        {
            Timed tm(tctx, st, SRE2_KIND_PASS2);
            e = f64 ? launch_pass2<double>(ws.scratch, N, slab, split, x0 + c0, (int)cs, ch.P,
                                           ws.part, se, spec, st)
                    : launch_pass2<float>(ws.scratch, N, slab, split, x0 + c0, (int)cs, ch.P,
                                          ws.part, se, spec, st);
        }
        if (e != hipSuccess) return SRE2_EHIP;
        {
            Timed tm(tctx, st, SRE2_KIND_AUX);
            e = launch_group_sum(ws.part, (int)cs, ch.P, Sx + c0, st);
        }
        if (e != hipSuccess) return SRE2_EHIP;
    }
    return SRE2_OK;
}

// Two-pass workspace of the shifts [x0, x0 + xc) with this scratch limit:
// *need = slab bytes and *need_part = column-group partials (doubles) for
// the largest chunk shape of its slab ranges.  Returns the largest chunk
// (shifts).
int64_t slab_need(int N, int form, bool pairs, int64_t x0, int64_t xc, size_t limit,
                  size_t* need, size_t* need_part) {
    const int elem = elem_bytes(work_dtype(form));
    *need = 0;
    *need_part = 0;
    int64_t cs_max = 0;
    SlabRange rg[2];
    const int nr = slab_ranges(N, form, pairs, x0, xc, rg);
    for (int i = 0; i < nr; ++i) {
        const Chunking c = chunking(N, form, rg[i].slab, rg[i].xc, limit);
        const size_t b = (size_t)c.cs * (size_t(1) << slab_bits(N, rg[i].slab)) * elem;
        *need = *need > b ? *need : b;
        *need_part = *need_part > (size_t)c.cs * c.P ? *need_part : (size_t)c.cs * c.P;
        cs_max = cs_max > c.cs ? cs_max : c.cs;
    }
    return cs_max;
}

// Grow the context's two-pass slab and partials for the shifts [x0, x0 + xc)
// and set ws.scratch, ws.part and ws.limit.  When the device cannot hold the
// slab, the chunks shrink (halving the limit for this call) down to one
// shift per chunk.  Chunking never changes a result bit.
// `pairs`: the call may take the row-pair slabs (the context allows them
// and the call reduces to M2).
int ctx_two_pass_ws(sre2_ctx* ctx, int N, int form, int64_t x0, int64_t xc, bool pairs,
                    Workspace* ws) {
    ws->pairs = pairs && ctx->row_pairs;
    if (N <= fused_max(form)) return SRE2_OK;
    size_t limit = ctx->scratch_limit, need = 0, need_part = 0;
    int rc;
    for (;;) {
        const int64_t cs_max = slab_need(N, form, ws->pairs, x0, xc, limit, &need, &need_part);
        rc = ensure(&ctx->scratch, &ctx->scratch_bytes, need);
        if (rc != SRE2_ENOMEM || cs_max <= 1) break;
        limit = need / 2;
    }
    if (rc) return rc;
    rc = ensure((void**)&ctx->part, &ctx->part_bytes, need_part * sizeof(double));
    if (rc) return rc;
    ws->scratch = ctx->scratch;
    ws->part = ctx->part;
    ws->limit = limit;
    return SRE2_OK;
}

// S_x for x in [x0, x0 + xc) into Sx (device, xc doubles).  The Hermitian
// forms route the shifts they cannot take (x = 0 fused, x < 2^L two-pass,
// or N too small) through the plain kernels of the same precision.
int shift_sums(sre2_ctx* tctx, const Workspace& ws, const void* work, int N, int form,
               int64_t x0, int64_t xc, double* Sx, const int* se, const Spec* spec,
               hipStream_t st) {
    if (fault_injected("launch")) return SRE2_EHIP;
    const bool f64 = is_f64(form);
    const int sp = split_kind(form);
    const int64_t x1 = x0 + xc;
    if (N <= fused_max(form)) {
        const bool herm = is_herm(form) && N >= herm_min(form);
        const int64_t split = herm ? (x0 > 1 ? x0 : (x1 < 1 ? x1 : 1)) : x1;  // plain: [x0, split)
        if (split > x0) {
            Timed tm(tctx, st, SRE2_KIND_SHIFT);
            const hipError_t e =
                f64 ? launch_shift_kernel<double>(work, N, false, false, x0, split - x0, Sx, se,
                                                  Pack{}, spec, st)
                    : launch_shift_kernel<float>(work, N, false, sp, x0, split - x0, Sx, se,
                                                 Pack{}, spec, st);
            if (e != hipSuccess) return SRE2_EHIP;
        }
        if (x1 > split) {
            Timed tm(tctx, st, SRE2_KIND_SHIFT);
            const hipError_t e =
                f64 ? launch_shift_kernel<double>(work, N, true, false, split, x1 - split,
                                                  Sx + (split - x0), se, Pack{}, spec, st)
                    : launch_shift_kernel<float>(work, N, true, false, split, x1 - split,
                                                 Sx + (split - x0), se, Pack{}, spec, st);
            if (e != hipSuccess) return SRE2_EHIP;
        }
        return SRE2_OK;
    }
    SlabRange rg[2];
    const int nr = slab_ranges(N, form, ws.pairs && spec == nullptr, x0, xc, rg);
    for (int i = 0; i < nr; ++i) {
        const int rc = two_pass(tctx, ws, work, N, form, rg[i].slab, rg[i].x0, rg[i].xc,
                                Sx + (rg[i].x0 - x0), se, spec, st);
        if (rc) return rc;
    }
    return SRE2_OK;
}

// Norm partials (and, for the split form, its scale exponent).
int norm_stage(sre2_ctx* tctx, const void* work, int N, int form, const Red& r, int nb,
               hipStream_t st) {
    Timed tm(tctx, st, SRE2_KIND_AUX);
    int rc = hip_status(launch_norm(work, work_dtype(form), int64_t(1) << N, nb, r.npart, r.nflag,
                                    Pack{}, st));
    if (!rc && is_split(form))
        rc = hip_status(launch_split_scale(r.npart, nb, r.se, Pack{}, st));
    return rc;
}

// The launch sequence of one evaluation on the buffers of ws: M2
// (spec == nullptr), or the general reduction of spec: M_alpha / M_1 in out,
// or the Pauli-spectrum counts in spec->hist (cleared here first).  S_x goes
// to `partials` when given, else to ws.sx; with sx_given the caller's
// `partials` already hold every S_x and only the norm, the fixed-order sum
// and the logarithm run.  tctx (may be null) only records per-launch timing.
int m2_launch(sre2_ctx* tctx, const Workspace& ws, const void* psi, int N, int dtype, int form,
              hipStream_t st, double* out, double* partials, const Spec* spec, bool sx_given) {
    const void* work = nullptr;
    int rc = stage_input(tctx, ws, psi, N, dtype, form, st, &work);
    if (rc) return rc;
    const int64_t n = int64_t(1) << N;
    const Red r = red_of(ws.red);
    const int nb = red_blocks(n);
    rc = norm_stage(tctx, work, N, form, r, nb, st);
    if (rc) return rc;
    double* Sx = partials ? partials : ws.sx;
    Spec sp{};
    if (spec) {
        sp = *spec;
        if (sp.kind == kRedHist) {
            Timed tm(tctx, st, SRE2_KIND_AUX);
            rc = hip_status(launch_norm_total(r.npart, nb, r.nrm, st));
            if (!rc) rc = hip_status(launch_zero_u64(sp.hist, sp.nbins, st));
            if (rc) return rc;
            sp.nrm = r.nrm;
        }
    }
    if (!sx_given) {
        rc = shift_sums(tctx, ws, work, N, form, 0, n, Sx, r.se, spec ? &sp : nullptr, st);
        if (rc) return rc;
    }
    {
        Timed tm(tctx, st, SRE2_KIND_AUX);
        rc = hip_status(launch_sum(Sx, n, 1, nb, r.spart, nullptr, Pack{}, st));
    }
    if (rc) return rc;
    Timed tm(tctx, st, SRE2_KIND_AUX);
    return hip_status(launch_final(r.spart, nb, r.npart, r.nflag, nb, N, out, Pack{},
                                   spec ? sp.kind : kRedQuartic, spec ? sp.alpha : 2.0, st));
}

// Grow the context's input copy and reduction buffers (and S_x when the
// caller passes no partials buffer) for a call of this shape.
int ctx_common_ws(sre2_ctx* ctx, int N, int dtype, int form, bool need_sx, Workspace* ws) {
    const int64_t n = int64_t(1) << N;
    const int wd = work_dtype(form);
    int rc;
    if (wd != dtype) {
        rc = ensure(&ctx->psi_work, &ctx->psi_work_bytes, (size_t)n * elem_bytes(wd));
        if (rc) return rc;
        ws->psi_work = ctx->psi_work;
    }
    rc = ensure((void**)&ctx->red, &ctx->red_bytes, red_doubles() * sizeof(double));
    if (rc) return rc;
    ws->red = ctx->red;
    if (need_sx) {
        rc = ensure((void**)&ctx->sx, &ctx->sx_bytes, (size_t)n * sizeof(double));
        if (rc) return rc;
        ws->sx = ctx->sx;
    }
    return SRE2_OK;
}

// One evaluation on the context's workspace (grown as needed).
int m2_one(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, hipStream_t st, double* out,
           double* partials, const Spec* spec = nullptr) {
    Workspace ws;
    int rc = ctx_common_ws(ctx, N, dtype, form, partials == nullptr, &ws);
    if (!rc) rc = ctx_two_pass_ws(ctx, N, form, 0, int64_t(1) << N, spec == nullptr, &ws);
    if (rc) return rc;
    return m2_launch(ctx, ws, psi, N, dtype, form, st, out, partials, spec, false);
}

// Up to kMaxPack states of one N <= fused_max(form) in packed launches: the
// same kernels, grids and reduction ranges as m2_one, with the grid's y index
// selecting the state, so every result is bitwise identical to a single call.
int m2_pack(sre2_ctx* ctx, const void* const* psi, int count, int N, int dtype, int form,
            double* const* outs, hipStream_t st) {
    const int wd = work_dtype(form);
    const int64_t n = int64_t(1) << N;
    Pack pk;
    pk.count = count;
    pk.N = N;
    int rc = ensure((void**)&ctx->pack_ws, &ctx->pack_ws_bytes,
                    (size_t)kMaxPack * pack_ws_doubles(N) * sizeof(double));
    if (rc) return rc;
    if (wd != dtype) {
        rc = ensure(&ctx->pack_work, &ctx->pack_work_bytes, (size_t)kMaxPack * n * elem_bytes(wd));
        if (rc) return rc;
    }
    for (int i = 0; i < count; ++i) {
        pk.ws[i] = ctx->pack_ws + (size_t)i * pack_ws_doubles(N);
        pk.out[i] = outs[i];
        if (wd == dtype) {
            pk.psi[i] = psi[i];
        } else {
            void* dst = (char*)ctx->pack_work + (size_t)i * n * elem_bytes(wd);
            Timed tm(ctx, st, SRE2_KIND_AUX);
            if (launch_convert(psi[i], dtype, dst, wd, n, st) != hipSuccess) return SRE2_EHIP;
            pk.psi[i] = dst;
        }
    }
    const bool f64 = is_f64(form);
    const int sp = split_kind(form);
    const bool herm = is_herm(form) && N >= herm_min(form);
    const int nb = red_blocks(n);
    {
        Timed tm(ctx, st, SRE2_KIND_AUX);
        if (launch_norm(nullptr, wd, n, nb, nullptr, nullptr, pk, st) != hipSuccess) return SRE2_EHIP;
        if (sp && launch_split_scale(nullptr, nb, nullptr, pk, st) != hipSuccess) return SRE2_EHIP;
    }
    if (fault_injected("launch")) return SRE2_EHIP;
    {
        Timed tm(ctx, st, SRE2_KIND_SHIFT);
        const int64_t plain_end = herm ? 1 : n;
        hipError_t e = f64 ? launch_shift_kernel<double>(nullptr, N, false, false, 0, plain_end,
                                                         nullptr, nullptr, pk, nullptr, st)
                           : launch_shift_kernel<float>(nullptr, N, false, sp, 0, plain_end,
                                                        nullptr, nullptr, pk, nullptr, st);
        if (e == hipSuccess && herm)
            e = f64 ? launch_shift_kernel<double>(nullptr, N, true, false, 1, n - 1, nullptr,
                                                  nullptr, pk, nullptr, st)
                    : launch_shift_kernel<float>(nullptr, N, true, false, 1, n - 1, nullptr,
                                                 nullptr, pk, nullptr, st);
        if (e != hipSuccess) return SRE2_EHIP;
    }
    Timed tm(ctx, st, SRE2_KIND_AUX);
    if (launch_sum(nullptr, n, 1, nb, nullptr, nullptr, pk, st) != hipSuccess) return SRE2_EHIP;
    if (launch_final(nullptr, nb, nullptr, nullptr, nb, N, nullptr, pk, kRedQuartic, 2.0, st) !=
        hipSuccess)
        return SRE2_EHIP;
    return SRE2_OK;
}

}  // namespace

namespace sre2 {
int ws_m2(const Workspace& ws, const void* psi, int N, int dtype, int form, hipStream_t st,
          double* out, double* partials) {
    return m2_launch(nullptr, ws, psi, N, dtype, form, st, out, partials, nullptr, false);
}
int ws_layout(int N, int dtype, int form, bool need_sx, size_t bytes, size_t* psi_work_off,
              size_t* sx_off, size_t* part_off, size_t* slab_off, size_t* limit) {
    const size_t n = size_t(1) << N;
    const auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = up(red_doubles() * sizeof(double));
    *psi_work_off = *sx_off = *part_off = *slab_off = 0;
    *limit = 0;
    if (work_dtype(form) != dtype) {
        *psi_work_off = off;
        off = up(off + n * (size_t)elem_bytes(work_dtype(form)));
    }
    if (need_sx) {
        *sx_off = off;
        off = up(off + n * sizeof(double));
    }
    if (off > bytes) return SRE2_ESCRATCH;
    if (N <= fused_max(form)) return SRE2_OK;
    // the largest chunks whose slab and partials fit what is left
    size_t lim = bytes - off, need = 0, need_part = 0;
    for (;;) {
        const int64_t cs = slab_need(N, form, true, 0, (int64_t)n, lim, &need, &need_part);
        const size_t pb = up(need_part * sizeof(double));
        if (off + pb + need <= bytes) {
            *part_off = off;
            *slab_off = off + pb;
            *limit = need;
            return SRE2_OK;
        }
        if (cs <= 1) return SRE2_ESCRATCH;
        lim = need / 2;
    }
}
int ctx_m2_one(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, hipStream_t st,
               double* out) {
    return m2_one(ctx, psi, N, dtype, form, st, out, nullptr);
}
int ctx_m2_pack(sre2_ctx* ctx, const void* const* psi, int count, int N, int dtype, int form,
                double* const* outs, hipStream_t st) {
    return m2_pack(ctx, psi, count, N, dtype, form, outs, st);
}
int ctx_fused_max(int form) { return fused_max(form); }
int ctx_reserve_pack(sre2_ctx* ctx, int N, int form) {
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    int rc = ensure((void**)&ctx->pack_ws, &ctx->pack_ws_bytes,
                    (size_t)kMaxPack * pack_ws_doubles(N) * sizeof(double));
    if (!rc)
        rc = ensure(&ctx->pack_work, &ctx->pack_work_bytes,
                    (size_t)kMaxPack * (size_t(1) << N) * elem_bytes(work_dtype(form)));
    return rc;
}
int ctx_validate_form(int N, int dtype, int form) {
    static const char kDummy = 0;
    sre2_ctx probe;
    return validate(&probe, &kDummy, N, dtype, form);
}
}  // namespace sre2

extern "C" {

int sre2_version(void) { return 100; }

const char* sre2_strerror(int status) {
    switch (status) {
        case SRE2_OK: return "success";
        case SRE2_EINVAL: return "invalid argument (null pointer, N out of range, bad count or range)";
        case SRE2_EDTYPE: return "unsupported dtype (expected SRE2_C64 or SRE2_C128)";
        case SRE2_EFORM: return "unsupported arithmetic form";
        case SRE2_ENORM: return "input state has zero norm or non-finite amplitudes";
        case SRE2_ENOMEM: return "device workspace allocation failed";
        case SRE2_EHIP: return "HIP runtime or kernel launch error";
        case SRE2_EBUSY: return "no free slot or memory budget";
        case SRE2_ECANCELLED: return "request cancelled";
        case SRE2_ENOTFOUND: return "unknown ticket";
        case SRE2_ESCRATCH:
            return "problem needs more device memory than the fixed scratch of the "
                   "allocation-free entry point";
        default: return "unknown status code";
    }
}

int sre2_create(sre2_ctx** out, int hip_device) {
    if (!out || hip_device < 0) return SRE2_EINVAL;
    sre2_ctx* c = new (std::nothrow) sre2_ctx();
    if (!c) return SRE2_ENOMEM;
    c->device = hip_device;
    *out = c;
    return SRE2_OK;
}

int sre2_destroy(sre2_ctx* ctx) {
    if (!ctx) return SRE2_OK;
    int rc = SRE2_OK;
    if (ctx->psi_work || ctx->sx || ctx->scratch || ctx->part || ctx->red || ctx->pack_ws ||
        ctx->pack_work) {
        DeviceGuard g(ctx->device);
        if (g.err != hipSuccess) rc = SRE2_EHIP;
        (void)hipDeviceSynchronize();
        void* bufs[] = {ctx->psi_work, ctx->sx,      ctx->scratch,  ctx->part,
                        ctx->red,      ctx->pack_ws, ctx->pack_work};
        for (void* b : bufs)
            if (b && hipFree(b) != hipSuccess) rc = SRE2_EHIP;
    }
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    delete ctx;
    return rc;
}

int sre2_set_scratch_limit(sre2_ctx* ctx, size_t bytes) {
    if (!ctx) return SRE2_EINVAL;
    ctx->scratch_limit = bytes;
    return SRE2_OK;
}

int sre2_row_bits(int N, int form) {
    if (N < 1 || N > SRE2_MAX_N || !form_ok(form)) return -1;
    if (N > (is_f64(form) ? max_n<double>() : max_n<float>())) return -1;
    if (N <= fused_max(form)) return 0;
    return row_bits(form, N - (is_herm(form) ? 1 : 0));
}

size_t sre2_workspace_bytes(int N, int dtype, int form) {
    if (N < 1 || N > SRE2_MAX_N || !dtype_ok(dtype) || !form_ok(form)) return 0;
    if (N > (is_f64(form) ? max_n<double>() : max_n<float>())) return 0;
    const size_t n = size_t(1) << N;
    size_t b = red_doubles() * sizeof(double) + n * sizeof(double);
    if (work_dtype(form) != dtype) b += n * (size_t)elem_bytes(work_dtype(form));
    if (N > fused_max(form)) {
        size_t slab = 0, part = 0;
        slab_need(N, form, true, 0, (int64_t)n, kDefaultScratchLimit, &slab, &part);
        b += slab + part * sizeof(double);
    }
    return b;
}

int sre2_m2(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, void* stream, double* out,
            double* partials) {
    int rc = validate(ctx, psi, N, dtype, form);
    if (rc) return rc;
    if (!out) return SRE2_EINVAL;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    return m2_one(ctx, psi, N, dtype, form, (hipStream_t)stream, out, partials);
}

int sre2_sre(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, double alpha,
             void* stream, double* out) {
    int rc = validate(ctx, psi, N, dtype, form);
    if (rc) return rc;
    if (!out || !(alpha > 0.0) || !std::isfinite(alpha)) return SRE2_EINVAL;
    if (alpha != 2.0 && is_split(form)) return SRE2_EFORM;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    if (alpha == 2.0) return m2_one(ctx, psi, N, dtype, form, (hipStream_t)stream, out, nullptr);
    Spec sp{};
    sp.kind = alpha == 1.0 ? kRedShannon : kRedPow;
    sp.alpha = alpha;
    return m2_one(ctx, psi, N, dtype, form, (hipStream_t)stream, out, nullptr, &sp);
}

int sre2_pauli_spectrum(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, int nbins,
                        void* stream, uint64_t* counts, double* out) {
    int rc = validate(ctx, psi, N, dtype, form);
    if (rc) return rc;
    if (!counts || !out || nbins < 2 || nbins > kMaxBins) return SRE2_EINVAL;
    if (is_split(form)) return SRE2_EFORM;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    Spec sp{};
    sp.kind = kRedHist;
    sp.nbins = nbins;
    sp.hist = reinterpret_cast<unsigned long long*>(counts);
    return m2_one(ctx, psi, N, dtype, form, (hipStream_t)stream, out, nullptr, &sp);
}

int sre2_moments(sre2_ctx* ctx, const void* psi, int N, int dtype, void* stream, double* out) {
    if (!ctx || !psi || !out || N < 1 || N > SRE2_MAX_N) return SRE2_EINVAL;
    if (!dtype_ok(dtype)) return SRE2_EDTYPE;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    const int rc = ensure((void**)&ctx->red, &ctx->red_bytes, red_doubles() * sizeof(double));
    if (rc) return rc;
    const int64_t n = int64_t(1) << N;
    Timed tm(ctx, (hipStream_t)stream, SRE2_KIND_AUX);
    return hip_status(launch_moments(psi, dtype == SRE2_C64 ? kC64 : kC128, n, red_blocks(n),
                                     ctx->red, out, (hipStream_t)stream));
}

int sre2_partials(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, int64_t x_begin,
                  int64_t x_count, void* stream, double* partials) {
    int rc = validate(ctx, psi, N, dtype, form);
    if (rc) return rc;
    const int64_t n = int64_t(1) << N;
    if (!partials || x_begin < 0 || x_count < 1 || x_begin > n || x_count > n - x_begin)
        return SRE2_EINVAL;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    const hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    rc = ctx_common_ws(ctx, N, dtype, form, false, &ws);
    if (!rc) rc = ctx_two_pass_ws(ctx, N, form, x_begin, x_count, true, &ws);
    if (rc) return rc;
    const void* work = nullptr;
    rc = stage_input(ctx, ws, psi, N, dtype, form, st, &work);
    if (rc) return rc;
    const Red r = red_of(ws.red);
    if (is_split(form)) {
        rc = norm_stage(ctx, work, N, form, r, red_blocks(n), st);
        if (rc) return rc;
    }
    return shift_sums(ctx, ws, work, N, form, x_begin, x_count, partials, r.se, nullptr, st);
}

int sre2_m2_from_partials(sre2_ctx* ctx, const void* psi, int N, int dtype, int form,
                          const double* partials, void* stream, double* out) {
    int rc = validate(ctx, psi, N, dtype, form);
    if (rc) return rc;
    if (!partials || !out) return SRE2_EINVAL;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    Workspace ws;
    rc = ctx_common_ws(ctx, N, dtype, form, false, &ws);
    if (rc) return rc;
    return m2_launch(ctx, ws, psi, N, dtype, form, (hipStream_t)stream, out,
                     const_cast<double*>(partials), nullptr, true);
}

int sre2_m2_batched(sre2_ctx* ctx, const void* const* psi_list, const int* N_list, int count,
                    int dtype, int form, void* stream, double* out) {
    if (!ctx || !psi_list || !N_list || !out || count < 1) return SRE2_EINVAL;
    for (int i = 0; i < count; ++i) {
        const int rc = validate(ctx, psi_list[i], N_list[i], dtype, form);
        if (rc) return rc;
    }
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    const hipStream_t st = (hipStream_t)stream;
    // states of one small N share packed launches; larger N run one by one
    for (int N = 1; N <= fused_max(form); ++N) {
        const void* psis[kMaxPack];
        double* outs[kMaxPack];
        int k = 0;
        for (int i = 0; i <= count; ++i) {
            if (i < count && N_list[i] == N) {
                psis[k] = psi_list[i];
                outs[k] = out + (size_t)SRE2_OUT_LEN * i;
                ++k;
            }
            if (k == kMaxPack || (i == count && k > 0)) {
                const int rc = m2_pack(ctx, psis, k, N, dtype, form, outs, st);
                if (rc) return rc;
                k = 0;
            }
        }
    }
    for (int i = 0; i < count; ++i) {
        if (N_list[i] <= fused_max(form)) continue;
        const int rc = m2_one(ctx, psi_list[i], N_list[i], dtype, form, st,
                              out + (size_t)SRE2_OUT_LEN * i, nullptr);
        if (rc) return rc;
    }
    return SRE2_OK;
}

int sre2_set_timing(sre2_ctx* ctx, int enable) {
    if (!ctx) return SRE2_EINVAL;
    ctx->timing = enable != 0;
    ctx->pending.clear();
    return SRE2_OK;
}

int sre2_timing_read(sre2_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx || !ms || !launches) return SRE2_EINVAL;
    for (int k = 0; k < SRE2_KIND_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    if (ctx->pending.empty()) return SRE2_OK;
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    if (hipEventSynchronize(ctx->events[ctx->pending.size() * 2 - 1]) != hipSuccess)
        return SRE2_EHIP;
    for (size_t i = 0; i < ctx->pending.size(); ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]) != hipSuccess)
            return SRE2_EHIP;
        ms[ctx->pending[i]] += t;
        launches[ctx->pending[i]] += 1;
    }
    ctx->pending.clear();
    return SRE2_OK;
}

int sre2_chunking(sre2_ctx* ctx, int N, int form, int64_t* shifts_per_chunk, int* groups) {
    if (!ctx || !shifts_per_chunk || !groups || N < 1 || N > SRE2_MAX_N || !form_ok(form))
        return SRE2_EINVAL;
    // the chunks of the high shifts x >= 2^L, most of an evaluation
    SlabRange rg[2];
    const int64_t n = int64_t(1) << N;
    const int nr = slab_ranges(N, form, ctx->row_pairs, 0, n, rg);
    const Chunking ch = chunking(N, form, rg[nr - 1].slab, n, ctx->scratch_limit);
    *shifts_per_chunk = ch.cs;
    *groups = ch.P;
    return SRE2_OK;
}

int64_t sre2_half_slab_first_shift(int N, int form) {
    if (N < 1 || N > SRE2_MAX_N || !form_ok(form)) return -1;
    if (N > (is_f64(form) ? max_n<double>() : max_n<float>())) return -1;
    const int64_t n = int64_t(1) << N;
    if (N <= fused_max(form)) return n;
    SlabRange rg[2];
    const int nr = slab_ranges(N, form, true, 0, n, rg);
    return rg[nr - 1].slab == kSlabFull ? n : rg[nr - 1].x0;
}

int sre2_set_row_pairs(sre2_ctx* ctx, int enable) {
    if (!ctx) return SRE2_EINVAL;
    ctx->row_pairs = enable != 0;
    return SRE2_OK;
}

}  // extern "C"
