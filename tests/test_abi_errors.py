"""The C ABI's error paths on the host, through the same ctypes binding the GPU tests use:
every entry point that takes a context rejects a null one with SKO_EINVAL (before any HIP
call), sko_strerror names every status, and sko_create reports a missing or invalid device
instead of failing later.  Runs without a GPU (on a GPU machine it also creates and destroys a
context)."""
import ctypes as C
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_16717_amd", "libsko.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsko.so not built")


@pytest.fixture(scope="module")
def B():
    from paper_2503_16717_amd import binding
    return binding


def test_null_context_is_rejected_by_every_entry_point(B):
    L = B._lib
    o = B.orth_opts()
    g = B.gmres_opts()
    A = B.sko_csr()
    R = (C.c_double * 4)()
    col = C.c_int32(0)
    assert L.sko_destroy(None) == B.SKO_EINVAL
    assert L.sko_set_stream(None, None) == B.SKO_EINVAL
    assert L.sko_orth_block(None, 8, 0, 2, None, 8, None, 8, None, 8, R, R, C.byref(o), C.byref(col)) == B.SKO_EINVAL
    assert L.sko_orth_block_noalloc(None, 8, 0, 2, None, 8, None, 8, None, 8, R, R, C.byref(o),
                                    C.byref(col)) == B.SKO_EINVAL
    assert L.sko_orth_blocks(None, 8, 1, 2, None, 8, None, 8, R, 2, C.byref(o), C.byref(col)) == B.SKO_EINVAL
    sk = B.make_sketch("sparse_sign", 16, 8, 0)
    assert L.sko_sketch_apply(None, 8, 2, None, 8, 0, C.byref(sk), R, 16) == B.SKO_EINVAL
    info = B.sko_gmres_info()
    assert L.sko_gmres(None, C.byref(A), None, None, C.byref(g), C.byref(info)) == B.SKO_EINVAL
    assert L.sko_gmres_batched(None, 1, C.byref(A), None, None, C.byref(g), C.byref(info)) == B.SKO_EINVAL
    assert L.sko_autotune_orth(None, 8, 1, 2, C.byref(o)) == B.SKO_EINVAL
    assert L.sko_profile_enable(None, 1) == B.SKO_EINVAL
    assert L.sko_profile_read(None, None, 0) == -B.SKO_EINVAL


def test_strerror_names_every_status(B):
    L = B._lib
    seen = set()
    for code in (B.SKO_OK, B.SKO_EINVAL, B.SKO_EDEVICE, B.SKO_ENOMEM, B.SKO_EBREAKDOWN, B.SKO_ENOCONV,
                 B.SKO_EUNSUPPORTED, B.SKO_ESCRATCH):
        msg = L.sko_strerror(code)
        assert isinstance(msg, bytes) and msg and msg != b"unknown status"
        seen.add(msg)
    assert len(seen) == 8
    assert L.sko_strerror(12345) == b"unknown status"


def test_create_reports_missing_or_invalid_device(B):
    L = B._lib
    h = C.c_void_p()
    assert L.sko_create(0, None, None) == B.SKO_EINVAL
    st = L.sko_create(0, None, C.byref(h))
    if st == B.SKO_OK:          # a device is present: the context works and is released
        assert h.value
        assert L.sko_destroy(h) == B.SKO_OK
        assert L.sko_create(1 << 20, None, C.byref(h)) == B.SKO_EINVAL
    else:                       # no device: the runtime error, and no context handed out
        assert st == B.SKO_EDEVICE
        assert not h.value
