"""The allocation-free entry point (su3hb_sweep_measure_static) against the
handle-based su3hb_sweep_measure on identical lattices: the links bit for
bit, the per-sweep plaquettes to rounding.  Two calls in a row on one GPU,
the second on a smaller lattice, so the shared static scratch must be
cleared and re-dimensioned by each call."""
import ctypes as C

import numpy as np
import pytest

import paper_0904_0642_amd as su3hb

pytestmark = pytest.mark.gpu

CASES = [  # extents, nlat, dlt mask, precision, betas, sweeps
    ((12, 12, 12, 12), 1, 0, su3hb.FP64_18, (5.9, 5.9), 3),
    ((6, 4, 4, 4), 2, 0b1111, su3hb.FP32_18, (5.6, 6.1), 2),
]


def test_static_scratch_sweeps_match_handle_path():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    su3hb.lib()
    for ext, nlat, mask, prec, (b0, b1), nsw in CASES:
        print(f"case static sweep ext={ext} nlat={nlat} prec={prec} sweeps={nsw}", flush=True)
        ref = su3hb.Lattice(ext, nlat=nlat, dlt_mask=mask, precision=prec, seed=5)
        ref.set_launch(256, 1, 2)          # the launch shape the static path uses
        tgt = su3hb.Lattice(ext, nlat=nlat, dlt_mask=mask, precision=prec, seed=5)
        assert np.array_equal(ref.get_links(), tgt.get_links())
        s_ref = ref.sweep_measure(b0, b1, n_hit=8, n_sweeps=nsw)
        series = torch.full((6 * nsw,), -1.0, dtype=torch.float64, device="cuda")
        p = su3hb.make_params(ext, nlat, mask, False, prec, su3hb.HOT, 5,
                              device_links=C.c_void_p(tgt.buffer.data_ptr()), device_bytes=tgt.buffer.numel(),
                              hip_stream=su3hb._torch_stream())
        su3hb.su3hb_sweep_measure_static(p, b0, b1, 8, nsw, 0, C.c_void_p(series.data_ptr()))
        torch.cuda.synchronize()
        s_tgt = series.cpu().numpy().reshape(nsw, 6)
        assert np.array_equal(ref.get_links(), tgt.get_links())
        assert np.array_equal(np.isnan(s_ref), np.isnan(s_tgt))
        good = ~np.isnan(s_ref)
        d = np.abs(s_ref[good] - s_tgt[good]) / np.maximum(1.0, np.abs(s_ref[good]))
        print(f"  max rel diff of the plaquette series {d.max():.2e}", flush=True)
        assert d.max() <= 1e-13
        ref.close()
        tgt.close()

