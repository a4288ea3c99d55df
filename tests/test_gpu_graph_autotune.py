"""HIP graph capture of the transforms and the library's autotuner.

A captured adjoint (or forward) is replayed several times; between replays
the program runs its own eager work, changes the input in place and
synchronises, and every replay is compared with the eager transform of the
input it saw. The autotuned plan must reproduce the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import nfft as onfft, metrics
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL_O2 = {"f64": 1e-12, "f32": 1e-5}


def _plan(x, M, m, prec, **kw):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] N={x.shape[0]} d={x.shape[1]} M={M} m={m} {prec} {kw}", flush=True)
    return Plan(x, M, 2.0, m, precision=prec, device="cuda:0", **kw)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nrhs,tuning", [(1, None), (4, {"rhs_per_group": 2}), (3, {"rhs_per_group": 1}),
                                         (1, {"spread_mode": 5}), (2, {"spread_mode": 7}),
                                         (9, {"spread_mode": 6, "item_nodes": 128})])
def test_graph_replays_match_eager(prec, nrhs, tuning):
    M, m = 64, 5
    x = wl.uniform_nodes(6000, 2, 80)
    N = x.shape[0]
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    p = _plan(x, M, m, prec, max_rhs=nrhs, tuning=tuning)
    p.set_weights((1.0 + 0.2 * wl.complex_normal(N, 81)) / N)
    f = torch.from_numpy(wl.complex_normal((nrhs, N), 82)).to("cuda", cdt)
    out = torch.empty((nrhs, M * M), dtype=cdt, device="cuda")
    g = p.graph_adjoint(f, out)
    fh = torch.from_numpy(wl.complex_normal((nrhs, M * M), 83)).to("cuda", cdt)
    fout = torch.empty((nrhs, N), dtype=cdt, device="cuda")
    gf = p.graph_forward(fh, fout)
    for rep in range(4):
        # new inputs in place, unrelated eager work, then the replay
        f.copy_(torch.from_numpy(wl.complex_normal((nrhs, N), 90 + rep)).to(cdt))
        fh.copy_(torch.from_numpy(wl.complex_normal((nrhs, M * M), 95 + rep)).to(cdt))
        out.fill_(float("nan"))
        fout.fill_(float("nan"))
        scratch = p.adjoint(f[:1].clone())
        torch.cuda.synchronize()
        g.replay()
        gf.replay()
        torch.cuda.synchronize()
        eager = p.adjoint(f.clone())
        eager_f = p.forward(fh.clone())
        torch.cuda.synchronize()
        # LDS atomics (float64 tiles) sum in no fixed order: equal up to rounding
        tol = 1e-14 if prec == "f64" else 1e-6
        assert metrics.rel_err(out.cpu().numpy(), eager.cpu().numpy()) <= tol, rep
        assert metrics.rel_err(fout.cpu().numpy(), eager_f.cpu().numpy()) <= tol, rep
        del scratch
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,M,nrhs", [(2, 64, 1), (2, 64, 4), (1, 512, 1), (3, 16, 1)])
def test_autotuned_plan_matches_oracle(prec, d, M, nrhs):
    from paper_2302_00414_amd.nfft import NfftError
    m = 5 if d < 3 else 4
    x = wl.uniform_nodes(5000, d, 100 + d)
    N = x.shape[0]
    p = _plan(x, M, m, prec, max_rhs=nrhs, tuning="auto")
    assert p.tuned_ms is not None and p.tuned_ms > 0
    t = p.tuning()
    print("[tuned]", t, p.tuned_ms, flush=True)
    assert t["rhs_per_group"] in (1, 2, 4, 8)
    if nrhs == 1 or d == 3:
        assert t["rhs_per_group"] == 1 or nrhs == 1
    F = wl.complex_normal((nrhs, N), 102)
    with pytest.raises(NfftError):
        p.adjoint(torch.from_numpy(F))  # weights are not set by the tuner
    w = (1.0 + 0.3 * wl.complex_normal(N, 103)) / N
    p.set_weights(w)
    got = p.adjoint(torch.from_numpy(F)).cpu().numpy()
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(nrhs):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2[prec]
    p.close()
