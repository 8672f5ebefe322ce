"""The C-ABI library loads, exports every function include/su3hb.h declares,
and rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_0904_0642_amd as su3hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "su3hb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(su3hb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for required in ("su3hb_init_lattice", "su3hb_sweep", "su3hb_plaquette", "su3hb_get_links",
                     "su3hb_set_links", "su3hb_free", "su3hb_last_error", "su3hb_batch_create",
                     "su3hb_autotune"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(su3hb.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing
    # and the binding marshals every one of them
    assert sorted(su3hb.exported_names()) == declared_functions()


def test_links_bytes():
    for prec, b in ((su3hb.FP64_18, 144), (su3hb.FP32_18, 72), (su3hb.FP32_12, 48), (su3hb.FP64_12, 96)):
        p = su3hb.make_params([4, 4, 4, 4], precision=prec)
        assert su3hb.su3hb_links_bytes(p) == 256 * 4 * b
    p = su3hb.make_params([24, 24, 24, 8], nlat=2, dlt_mask=15, precision=su3hb.FP32_18)
    assert su3hb.su3hb_links_bytes(p) == 2 * 24 ** 3 * 8 * 4 * 72
    # each slab of V/2 links is stored as whole tiles of 64: 6 x 4 has V/2 = 12
    p = su3hb.make_params([6, 4], precision=su3hb.FP64_18)
    assert su3hb.su3hb_links_bytes(p) == 2 * 2 * 64 * 144
    p = su3hb.make_params([6, 6, 4], nlat=2, dlt_mask=7, precision=su3hb.FP32_12)
    assert su3hb.su3hb_links_bytes(p) == 2 * 3 * 2 * 128 * 48


@pytest.mark.parametrize("kw,frag", [
    (dict(extents=[3, 4, 4, 4]), "even"),
    (dict(extents=[4]), "nd"),
    (dict(extents=[4] * 7), "nd"),
    (dict(extents=[4, 4], nlat=3), "nlat"),
    (dict(extents=[4, 4], dlt_mask=1), "nlat = 2"),
    (dict(extents=[4, 4], lat2test=True), "nlat = 2"),
    (dict(extents=[4, 4], nlat=2, dlt_mask=4), "dlt_mask"),
    (dict(extents=[4, 4], precision=7), "precision"),
    (dict(extents=[4, 4], start=9), "start"),
    (dict(extents=[0, 4]), "even"),
])
def test_init_rejects_bad_parameters(kw, frag):
    ext = kw.pop("extents")
    p = su3hb.make_params(ext, **kw)
    with pytest.raises(su3hb.SU3HBError) as ei:
        su3hb.su3hb_init_lattice(p)
    assert ei.value.code == su3hb.EINVAL
    assert frag in str(ei.value)


def test_null_handles_are_rejected():
    lib = su3hb.lib()
    assert lib.su3hb_sweep(None, 6.0, 6.0, 8, 1, None) == su3hb.EINVAL
    assert lib.su3hb_plaquette(None, 6.0, 6.0, None) == su3hb.EINVAL
    assert lib.su3hb_get_links(None, None, 0) == su3hb.EINVAL
    assert lib.su3hb_batch_sweep(None, 8, 1, 0, None) == su3hb.EINVAL
    assert "NULL" in su3hb.last_error() or "batch" in su3hb.last_error()
    lib.su3hb_free(None)
    lib.su3hb_batch_free(None)


def test_batch_rejects_bad_replicas():
    with pytest.raises(su3hb.SU3HBError):
        su3hb.su3hb_batch_create(4, [((4, 4, 4, 3), 6.0, 1, su3hb.HOT)], su3hb.FP32_18)
    with pytest.raises(su3hb.SU3HBError):
        su3hb.su3hb_batch_create(4, [], su3hb.FP32_18)


@pytest.mark.parametrize("ext", [(256, 256, 256, 64), (182, 182, 182, 182)])
def test_batch_rejects_replica_beyond_32bit_link_ids(ext):
    # fewer than 2^32 sites but at least 2^32 links: the 32-bit Philox link id
    # would wrap (colliding random streams), so the replica is refused before
    # any device call (this host has no GPU)
    assert int(np.prod(ext)) < 2 ** 32 <= 4 * int(np.prod(ext))
    with pytest.raises(su3hb.SU3HBError) as ei:
        su3hb.su3hb_batch_create(4, [((4, 4, 4, 4), 6.0, 1, su3hb.HOT), (ext, 6.0, 2, su3hb.HOT)],
                                 su3hb.FP32_12)
    assert ei.value.code == su3hb.EINVAL
    assert "replica 1" in str(ei.value) and "2^32 links" in str(ei.value)


def test_init_rejects_beyond_32bit_link_ids():
    p = su3hb.make_params([256, 256, 256, 64], precision=su3hb.FP32_12)
    with pytest.raises(su3hb.SU3HBError) as ei:
        su3hb.su3hb_init_lattice(p)
    assert ei.value.code == su3hb.EINVAL and "2^32 links" in str(ei.value)


def test_no_cpu_fallback_in_package():
    # the product path never imports the oracle
    pkg = os.path.join(ROOT, "paper_0904_0642_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt


def test_static_scratch_rejects_oversized_measurement():
    # su3hb_sweep_measure_static on 128^4: the per-block partial sums of the
    # measurement exceed the static scratch; refused before any device work
    # (a dummy, aligned device pointer that is never dereferenced)
    p = su3hb.make_params([128, 128, 128, 128], precision=su3hb.FP32_12, device_links=C.c_void_p(1 << 20),
                          device_bytes=1 << 40)
    with pytest.raises(su3hb.SU3HBError) as ei:
        su3hb.su3hb_sweep_measure_static(p, 6.0, 6.0, 8, 1, 0, C.c_void_p(1 << 21))
    assert ei.value.code == su3hb.EINVAL and "static scratch" in str(ei.value)
