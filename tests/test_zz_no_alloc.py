"""The entry point that allocates nothing (hpm_solve_noalloc) against the one-shot solve it is a
variant of (hpm_solve), called through the C ABI: two calls in a row on the shared scratch region,
the second with a smaller input, each compared with hpm_solve on the same inputs. The bar is the
parity bar (FP64 1e-10 relative per particle, FP32 1e-5 relative RMS in potential); the two run
the same kernels in the same order, so the results are expected to be identical."""
import ctypes

import numpy as np
import pytest

from synth import plummer_sphere, uniform_cube
from tests.hpmcase import log, rel_each_max, rel_rms

pytestmark = pytest.mark.gpu


def _call(fn, prob, arrays, torch, dt):
    from paper_1906_10734_amd import hpm
    n = arrays[0].numel()
    out = [torch.full((n,), float("nan"), dtype=dt, device="cuda") for _ in range(4)]
    c = prob.c()
    st = fn(ctypes.byref(c), n, *(a.data_ptr() for a in arrays), *(o.data_ptr() for o in out),
            torch.cuda.current_stream().cuda_stream)
    assert st == 0, hpm._lib.hpm_last_error().decode()
    torch.cuda.synchronize()
    return [o.double().cpu().numpy() for o in out]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_solve_equals_solve(prec):
    import torch
    from paper_1906_10734_amd import hpm
    lib = hpm._lib
    dt = torch.float32 if prec == "f32" else torch.float64
    npdt = np.float32 if prec == "f32" else np.float64
    cases = [(plummer_sphere(8000, 31, a=0.08),
              hpm.Problem(ng=6, precision=prec, leaf_capacity=32, max_depth=10, softening=1e-3)),
             (uniform_cube(4096, 1000),
              hpm.Problem(ng=4, precision=prec, uniform_depth=3, softening=1e-3))]
    for p, prob in cases:  # the second call is the smaller input
        q = p.astype(npdt)
        arrays = [torch.tensor(a, dtype=dt, device="cuda") for a in (q.x, q.y, q.z, q.m)]
        ref = _call(lib.hpm_solve, prob, arrays, torch, dt)
        got = _call(lib.hpm_solve_noalloc, prob, arrays, torch, dt)
        acc_r = np.stack(ref[1:], 1)
        acc_g = np.stack(got[1:], 1)
        same = all(np.array_equal(a, b) for a, b in zip(ref, got))
        log(f"[noalloc] {prec} n={q.n} ng={prob.ng}: identical={same} "
            f"phi {rel_rms(got[0], ref[0]):.2e} acc {rel_rms(acc_g, acc_r):.2e}")
        assert np.isfinite(got[0]).all() and np.isfinite(acc_g).all()
        if prec == "f64":
            assert rel_each_max(got[0], ref[0]) < 1e-10
            assert rel_each_max(acc_g, acc_r) < 1e-10
        else:
            assert rel_rms(got[0], ref[0]) < 1e-5
            assert rel_rms(acc_g, acc_r) < 1e-4


def test_noalloc_rejects_problems_beyond_the_region():
    import torch
    from paper_1906_10734_amd import hpm
    lib = hpm._lib
    prob = hpm.Problem(ng=6, precision="f64", leaf_capacity=8, max_depth=10).c()
    dummy = ctypes.c_void_p(1)
    st = lib.hpm_solve_noalloc(ctypes.byref(prob), 2 ** 20, *([dummy] * 8),
                               torch.cuda.current_stream().cuda_stream)
    assert st == 4  # HPM_ERR_NO_MEMORY, before any device work
    assert b"MiB" in lib.hpm_last_error()
