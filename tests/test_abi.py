"""C-ABI checks that need no GPU: the library loads, exports every function
include/sre2.h declares, and rejects bad arguments on the host before any
device work (no compute calls are made here)."""
import ctypes

import pytest

import paper_2512_24685_amd as sre2

FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


@pytest.fixture(scope="module")
def L():
    return sre2.lib()


@pytest.fixture()
def ctx(L):
    c = sre2.Context(0)
    yield c
    c.close()


def test_exports_every_header_function(L):
    names = sre2.header_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n


def test_version_and_strerror(L):
    assert L.sre2_version() >= 100
    for code in range(0, -11, -1):
        s = L.sre2_strerror(code)
        assert s and s != b"unknown status code"
    assert L.sre2_strerror(12345) == b"unknown status code"


def test_create_destroy_without_device_work(L):
    p = ctypes.c_void_p()
    assert L.sre2_create(None, 0) == sre2.EINVAL
    assert L.sre2_create(ctypes.byref(p), -1) == sre2.EINVAL
    assert L.sre2_create(ctypes.byref(p), 0) == sre2.OK
    assert L.sre2_set_scratch_limit(p, 1 << 20) == sre2.OK
    assert L.sre2_destroy(p) == sre2.OK
    assert L.sre2_destroy(None) == sre2.OK
    assert L.sre2_set_scratch_limit(None, 1) == sre2.EINVAL


def test_m2_argument_validation(L, ctx):
    out = FAKE
    h = ctx.handle
    assert L.sre2_m2(None, FAKE, 10, 0, 0, None, out, None) == sre2.EINVAL
    assert L.sre2_m2(h, None, 10, 0, 0, None, out, None) == sre2.EINVAL
    assert L.sre2_m2(h, FAKE, 0, 0, 0, None, out, None) == sre2.EINVAL
    assert L.sre2_m2(h, FAKE, sre2.MAX_N + 1, 0, 0, None, out, None) == sre2.EINVAL
    assert L.sre2_m2(h, FAKE, 10, 7, 0, None, out, None) == sre2.EDTYPE
    assert L.sre2_m2(h, FAKE, 10, 0, 99, None, out, None) == sre2.EFORM
    assert L.sre2_m2(h, FAKE, 10, 0, 0, None, None, None) == sre2.EINVAL


def test_sre_and_spectrum_argument_validation(L, ctx):
    h = ctx.handle
    nan, inf = float("nan"), float("inf")
    assert L.sre2_sre(None, FAKE, 10, 0, 0, 3.0, None, FAKE) == sre2.EINVAL
    assert L.sre2_sre(h, FAKE, 10, 0, 0, 3.0, None, None) == sre2.EINVAL
    for a in (0.0, -1.0, nan, inf):
        assert L.sre2_sre(h, FAKE, 10, 0, 0, a, None, FAKE) == sre2.EINVAL
    assert L.sre2_sre(h, FAKE, 10, 7, 0, 3.0, None, FAKE) == sre2.EDTYPE
    assert L.sre2_sre(h, FAKE, 10, 0, sre2.FORMS["split16"], 3.0, None, FAKE) == sre2.EFORM
    assert L.sre2_sre(h, FAKE, 10, 0, sre2.FORMS["split16"], 1.0, None, FAKE) == sre2.EFORM
    assert L.sre2_sre(h, FAKE, 10, 0, sre2.FORMS["splitbf16"], 3.0, None, FAKE) == sre2.EFORM
    sp = L.sre2_pauli_spectrum
    assert sp(h, FAKE, 10, 0, 0, 1, None, FAKE, FAKE) == sre2.EINVAL
    assert sp(h, FAKE, 10, 0, 0, 65, None, FAKE, FAKE) == sre2.EINVAL
    assert sp(h, FAKE, 10, 0, 0, 16, None, None, FAKE) == sre2.EINVAL
    assert sp(h, FAKE, 10, 0, 0, 16, None, FAKE, None) == sre2.EINVAL
    assert sp(h, FAKE, 0, 0, 0, 16, None, FAKE, FAKE) == sre2.EINVAL
    assert sp(h, FAKE, 10, 0, sre2.FORMS["split16"], 16, None, FAKE, FAKE) == sre2.EFORM
    assert sp(h, FAKE, 10, 0, sre2.FORMS["splitbf16"], 16, None, FAKE, FAKE) == sre2.EFORM


def test_partials_argument_validation(L, ctx):
    h = ctx.handle
    assert L.sre2_partials(h, FAKE, 4, 0, 0, 0, 17, None, FAKE) == sre2.EINVAL
    assert L.sre2_partials(h, FAKE, 4, 0, 0, -1, 2, None, FAKE) == sre2.EINVAL
    assert L.sre2_partials(h, FAKE, 4, 0, 0, 15, 2, None, FAKE) == sre2.EINVAL
    assert L.sre2_partials(h, FAKE, 4, 0, 0, 0, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_partials(h, FAKE, 4, 0, 0, 0, 4, None, None) == sre2.EINVAL
    assert L.sre2_partials(h, FAKE, 4, 3, 0, 0, 4, None, FAKE) == sre2.EDTYPE
    assert L.sre2_moments(None, FAKE, 4, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_moments(h, None, 4, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_moments(h, FAKE, 4, 0, None, None) == sre2.EINVAL
    assert L.sre2_moments(h, FAKE, 0, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_moments(h, FAKE, 27, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_moments(h, FAKE, 4, 2, None, FAKE) == sre2.EDTYPE


def test_batched_argument_validation(L, ctx):
    h = ctx.handle
    ptrs = (ctypes.c_void_p * 2)(0x10000, 0x20000)
    Ns = (ctypes.c_int * 2)(8, 40)
    assert L.sre2_m2_batched(h, ptrs, Ns, 0, 0, 0, None, FAKE) == sre2.EINVAL
    assert L.sre2_m2_batched(h, ptrs, Ns, 2, 0, 0, None, FAKE) == sre2.EINVAL  # N=40
    Ns[1] = 9
    assert L.sre2_m2_batched(h, ptrs, Ns, 2, 0, 99, None, FAKE) == sre2.EFORM
    assert L.sre2_m2_batched(h, ptrs, Ns, 2, 0, 0, None, None) == sre2.EINVAL


def test_workspace_bytes(L):
    assert L.sre2_workspace_bytes(0, 0, 0) == 0
    assert L.sre2_workspace_bytes(10, 9, 0) == 0
    small = L.sre2_workspace_bytes(10, sre2.C64, sre2.FORMS["fp32"])
    big = L.sre2_workspace_bytes(20, sre2.C64, sre2.FORMS["fp32"])
    assert 0 < small < big
    # FP64 on complex64 input stages a widened copy
    assert (L.sre2_workspace_bytes(12, sre2.C64, sre2.FORMS["fp64"])
            > L.sre2_workspace_bytes(12, sre2.C128, sre2.FORMS["fp64"]))


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        sre2.m2(torch.zeros(16, dtype=torch.complex64))


def test_server_argument_validation(L):
    p = ctypes.c_void_p()
    assert L.sre2_server_create(None, 0, 0, 1 << 30, 8) == sre2.EINVAL
    assert L.sre2_server_create(ctypes.byref(p), -1, 0, 1 << 30, 8) == sre2.EINVAL
    assert L.sre2_server_create(ctypes.byref(p), 0, 0, 1 << 30, 0) == sre2.EINVAL
    assert L.sre2_server_create(ctypes.byref(p), 0, 0, 1024, 8) == sre2.EINVAL
    assert L.sre2_server_create(ctypes.byref(p), 0, 99, 1 << 30, 8) == sre2.EFORM
    t = ctypes.c_uint64()
    st = ctypes.c_int()
    assert L.sre2_server_submit(None, FAKE, 8, 0, 0, ctypes.byref(t)) == sre2.EINVAL
    assert L.sre2_server_poll(None, 1, ctypes.byref(st), None, None) == sre2.EINVAL
    assert L.sre2_server_cancel(None, 1) == sre2.EINVAL
    assert L.sre2_server_drain(None, 1.0) == sre2.EINVAL
    assert L.sre2_server_stats(None, None, 0) == sre2.EINVAL
    assert L.sre2_server_destroy(None) == sre2.OK


def test_sim_argument_validation(L):
    p = ctypes.c_void_p()
    assert L.sre2_sim_create(None, 0, 8) == sre2.EINVAL
    assert L.sre2_sim_create(ctypes.byref(p), -1, 8) == sre2.EINVAL
    assert L.sre2_sim_create(ctypes.byref(p), 0, 1) == sre2.EINVAL
    assert L.sre2_sim_create(ctypes.byref(p), 0, 27) == sre2.EINVAL
    assert L.sre2_sim_destroy(None) == sre2.OK
    assert L.sre2_sim_product_state(None, None, None) == sre2.EINVAL
    assert L.sre2_sim_apply_gates(None, None, None, 0) == sre2.EINVAL
    assert L.sre2_sim_tfim_step(None, 1.0, 1.0, 1.0, 0.1) == sre2.EINVAL
    assert L.sre2_sim_state(None, 0, FAKE) == sre2.EINVAL
    assert L.sre2_sim_run_tfim(None, FAKE, 1.0, 1.0, 1.0, 0.1, 3, 0, None) == sre2.EINVAL
    assert L.sre2_sim_run_circuit(None, FAKE, None, None, 0, 3, 0, None) == sre2.EINVAL


def test_row_bits_query(L):
    f = sre2.FORMS
    assert L.sre2_row_bits(14, f["fp32"]) == 0  # fused
    assert L.sre2_row_bits(20, f["fp32"]) == 12
    assert L.sre2_row_bits(23, f["fp32"]) == 13 and L.sre2_row_bits(24, f["fp32"]) == 14
    assert L.sre2_row_bits(24, f["fp32h"]) == 13  # slab of N - 1 bits
    assert L.sre2_row_bits(22, f["fp64"]) == 12 and L.sre2_row_bits(24, f["fp64"]) == 13
    assert L.sre2_row_bits(0, f["fp32"]) == -1 and L.sre2_row_bits(20, 99) == -1
    assert L.sre2_row_bits(25, f["fp64"]) == -1  # beyond the FP64 maximum


def test_workspace_bytes_covers_default_chunks(L):
    """sre2_workspace_bytes sizes the slab with the default scratch limit of a
    fresh context: at least the slab of one default chunk (shifts per chunk
    from sre2_chunking: half slabs for the Hermitian-pair forms and the row
    pairs of the plain FP32 / FP64 forms) for every form."""
    ctx = sre2.Context(0)
    try:
        for form, herm in (("fp32", True), ("fp32h", True), ("split16", True),
                           ("fp64", True), ("fp64h", True)):
            elem = 16 if form.startswith("fp64") else 8
            for N in (15, 18, 20, 22, 24):
                if N > 24 and form.startswith("fp64"):
                    continue
                cs, P = ctx.chunking(N, form)
                ns = N - (1 if herm else 0)
                slab = cs * (1 << ns) * elem
                got = L.sre2_workspace_bytes(N, sre2.C64, sre2.FORMS[form])
                assert got >= slab + cs * P * 8 + (1 << N) * 8, (form, N, got, slab)
                # and no more than a full default scratch limit beyond the rest
                assert got <= (32 << 30) + (1 << N) * 8 * 4 + (1 << 20), (form, N, got)
    finally:
        ctx.close()


def test_default_context_per_stream():
    """Calls without a ctx on different streams get different contexts."""
    a = sre2.context(0, 111)
    b = sre2.context(0, 222)
    assert a is not b
    assert sre2.context(0, 111) is a


def test_noalloc_argument_validation(L):
    """sre2_m2_noalloc rejects bad arguments and problems larger than its
    fixed scratch on the host, before touching a device."""
    f = sre2.FORMS
    assert L.sre2_m2_noalloc(-1, FAKE, 10, 0, 0, None, FAKE, None) == sre2.EINVAL
    assert L.sre2_m2_noalloc(0, None, 10, 0, 0, None, FAKE, None) == sre2.EINVAL
    assert L.sre2_m2_noalloc(0, FAKE, 10, 0, 0, None, None, None) == sre2.EINVAL
    assert L.sre2_m2_noalloc(0, FAKE, 0, 0, 0, None, FAKE, None) == sre2.EINVAL
    assert L.sre2_m2_noalloc(0, FAKE, 10, 5, 0, None, FAKE, None) == sre2.EDTYPE
    assert L.sre2_m2_noalloc(0, FAKE, 10, 0, 99, None, FAKE, None) == sre2.EFORM
    # beyond the documented limits (complex64 input, no partials buffer)
    assert L.sre2_m2_noalloc(0, FAKE, 21, sre2.C64, f["fp32"], None, FAKE, None) == sre2.ESCRATCH
    assert L.sre2_m2_noalloc(0, FAKE, 20, sre2.C64, f["fp64"], None, FAKE, None) == sre2.ESCRATCH
    assert L.sre2_m2_noalloc(0, FAKE, 26, sre2.C64, f["fp32h"], None, FAKE, None) == sre2.ESCRATCH
    assert L.sre2_strerror(sre2.ESCRATCH) != b"unknown status code"


def test_row_pairs_setting_sets_the_chunk_shape():
    """sre2_set_row_pairs: host-only; with row pairs the plain and split
    forms chunk the shifts above 2^L in half slabs (twice the shifts per
    chunk at the same scratch limit), without them in full slabs; the
    Hermitian-pair forms keep their own half slabs either way."""
    L = sre2.lib()
    assert L.sre2_set_row_pairs(None, 1) == sre2.EINVAL
    ctx = sre2.Context(0)
    try:
        for form in ("fp32", "fp64", "split16", "splitbf16"):
            cs_on, P_on = ctx.chunking(22, form)
            ctx.set_row_pairs(False)
            cs_off, P_off = ctx.chunking(22, form)
            ctx.set_row_pairs(True)
            assert cs_on == 2 * cs_off and P_on == P_off
        cs_h, _ = ctx.chunking(22, "fp32h")
        ctx.set_row_pairs(False)
        assert ctx.chunking(22, "fp32h")[0] == cs_h
    finally:
        ctx.close()


def test_half_slab_first_shift():
    """Where the half slabs start (host-only): 2^L for the row pairs and the
    Hermitian pair at N = 20, 2^(L + 5) for the FP32 row pairs at N = 22 and
    24 (half-LDS pass-2 tiles whose lowest register row bit is row bit 5),
    2^N for fused sizes and -1 for bad arguments."""
    L = sre2.lib()
    assert sre2.half_slab_first_shift(20, "fp32") == 1 << 12
    assert sre2.half_slab_first_shift(20, "fp32h") == 1 << 12
    assert sre2.half_slab_first_shift(20, "fp64") == 1 << 11
    assert sre2.half_slab_first_shift(22, "fp32") == 1 << 17
    assert sre2.half_slab_first_shift(24, "fp32") == 1 << 19
    assert sre2.half_slab_first_shift(14, "fp32") == 1 << 14
    assert L.sre2_half_slab_first_shift(0, sre2.FORMS["fp32"]) == -1
    for N in range(15, 25):
        for form in ("fp32", "split16", "fp32h"):
            f = sre2.half_slab_first_shift(N, form)
            assert (1 << sre2.row_bits(N, form)) <= f < (1 << N) and f & (f - 1) == 0
