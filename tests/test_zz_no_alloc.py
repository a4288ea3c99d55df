"""nfft_adjoint_scratch, the adjoint whose intermediate buffers live in the
library's file-scope scratch array instead of the plan's workspace, against
nfft_adjoint on the same plan, through the C ABI: two calls in a row, the
second on a smaller input with most tiles empty (so stale data the first call
left in the scratch array must be cleared), and the refusal of a plan whose
buffers exceed the array."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import metrics
from paper_2302_00414_amd import _lib
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# two launches of the same kernels: float32 sums in a fixed order (same
# bits); float64 spreading adds with LDS atomics (rounding order only)
TOL = {"f32": 0.0, "f64": 1e-13}


def _call(name, plan, f, out, nrhs):
    lib = _lib.load()
    st = getattr(lib, name)(plan.handle, ctypes.c_void_p(f.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), nrhs,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(x, M, m, prec, nrhs, seed, tuning=None):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] N={x.shape[0]} M={M} m={m} {prec} rhs={nrhs} tuning={tuning}", flush=True)
    N = x.shape[0]
    p = Plan(x, M, 2.0, m, precision=prec, max_rhs=nrhs, device="cuda:0", tuning=tuning)
    p.set_weights((1.0 + 0.3 * wl.complex_normal(N, seed)) / N)
    f = torch.from_numpy(wl.complex_normal((nrhs, N), seed + 1)).to("cuda:0", p.cdtype)
    ws = torch.empty((nrhs, M * M), dtype=p.cdtype, device="cuda:0")
    sc = torch.full((nrhs, M * M), float("nan"), dtype=p.cdtype, device="cuda:0")
    assert _call("nfft_adjoint", p, f, ws, nrhs) == _lib.NFFT_OK
    assert _call("nfft_adjoint_scratch", p, f, sc, nrhs) == _lib.NFFT_OK, \
        _lib.load().nfft_last_error(p.handle)
    torch.cuda.synchronize()
    a, b = ws.cpu().numpy(), sc.cpu().numpy()
    p.close()
    return a, b


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("tuning", [None, {"spread_mode": 5}])
def test_scratch_adjoint_matches_workspace_adjoint(prec, tuning):
    # first: the polar 512 x 512 set at M = 256, m = 6 (corner tiles empty)
    x1 = wl.polar_nodes(512, 512)
    a1, b1 = _case(x1, 256, 6, prec, 1, 400, tuning)
    # second, smaller: 3000 nodes in one quadrant (three quarters of the
    # tiles empty, where the first call left its partial sums), 2 rhs
    x2 = -0.5 + 0.5 * (wl.uniform_nodes(3000, 2, 401) + 0.5)
    a2, b2 = _case(x2, 64, 4, prec, 2, 402, tuning)
    for a, b in ((a1, b1), (a2, b2)):
        assert np.all(np.isfinite(b))
        for r in range(a.shape[0]):
            err = metrics.rel_err(b[r], a[r])
            print(f"scratch vs workspace ({prec}): {err:.3e}", flush=True)
            assert err <= TOL[prec], r


def test_scratch_adjoint_with_gather_spreading():
    """Spread mode 6 through the scratch array (its grid where the tile
    partials would be, its unit partials and node-major samples after the
    FFT buffers): a crowded node set whose densest tile is cut into several
    units, then a smaller one, each against nfft_adjoint on the same plan
    (float32, same bits)."""
    rng = np.random.default_rng(405)
    x1 = np.concatenate([wl.uniform_nodes(6000, 2, 406),
                         0.01 * rng.standard_normal((3000, 2))])
    a1, b1 = _case(x1, 64, 6, "f32", 5, 407, {"spread_mode": 6, "item_nodes": 256})
    x2 = -0.5 + 0.5 * (wl.uniform_nodes(3000, 2, 408) + 0.5)
    a2, b2 = _case(x2, 32, 4, "f32", 2, 409, {"spread_mode": 6})
    for a, b in ((a1, b1), (a2, b2)):
        assert np.all(np.isfinite(b))
        for r in range(a.shape[0]):
            assert metrics.rel_err(b[r], a[r]) <= TOL["f32"], r


def test_scratch_refuses_oversized_plan():
    """d = 3, M = 64 (4096 tiles of 16^3 padded cells): the tile partials
    alone exceed the scratch array; the call fails before launching and
    leaves the output untouched."""
    from paper_2302_00414_amd.nfft import Plan
    x = wl.uniform_nodes(2000, 3, 403)
    p = Plan(x, 64, 2.0, 4, precision="f32", device="cuda:0")
    p.set_weights(np.full(2000, 1.0 / 2000))
    f = torch.from_numpy(wl.complex_normal(2000, 404)).to("cuda:0", torch.complex64)
    out = torch.full((64 ** 3,), 7.0, dtype=torch.complex64, device="cuda:0")
    assert _call("nfft_adjoint_scratch", p, f, out, 1) == _lib.NFFT_EUNSUPPORTED
    assert b"scratch" in _lib.load().nfft_last_error(p.handle)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    p.close()
