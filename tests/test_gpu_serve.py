"""The request loop on the GPU: results are the same alone and in a mix of
concurrent, batched requests, and match the oracle."""
import numpy as np
import pytest
import torch

from oracle import ndft, metrics
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def test_alone_vs_mix_and_oracle():
    from paper_2302_00414_amd.serve import Server
    print("[case] server alone-vs-mix", flush=True)
    sets = {
        "u32": (wl.uniform_nodes(3000, 2, 1), 32),
        "p64": (wl.polar_nodes(64, 64), 64),
        "s64": (wl.spiral_nodes(5000, 64), 64),
    }
    srv = Server(8 << 30, max_slots=3, max_batch_rhs=8).start()
    weights = {}
    for k, (x, M) in sets.items():
        w = (1.0 + 0.2 * wl.complex_normal(x.shape[0], 7)) / x.shape[0]
        weights[k] = w
        srv.register(k, x, M, 2.0, 6, w)
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(24):
        k = list(sets)[rng.integers(3)]
        nrhs = int(rng.integers(1, 4))
        f = wl.complex_normal((nrhs, sets[k][0].shape[0]), 100 + i)
        reqs.append((k, f, torch.from_numpy(f).to("cuda:0", torch.complex64)))
    alone = []
    for k, _, fd in reqs:
        alone.append(srv.submit(k, fd).result(timeout=60).cpu().numpy())
    b0 = srv.batches
    futs = [srv.submit(k, fd) for k, _, fd in reqs]
    mix = [f.result(timeout=60).cpu().numpy() for f in futs]
    batches_mix = srv.batches - b0
    st = srv.stats()
    srv.close()
    assert batches_mix < len(reqs)            # requests were fused into shared batches
    for a, b in zip(alone, mix):
        assert metrics.rel_err(b, a) <= 1e-6
    # every node set against the exact weighted sums at sampled frequencies
    seen = set()
    for (k, f, _), a in zip(reqs, alone):
        if k in seen:
            continue
        seen.add(k)
        x, M = sets[k]
        K = ndft.index_set(M, 2)
        sel = np.arange(0, M * M, 37)
        exact = ndft.adjoint_at(x, weights[k][None, :] * f, K[sel])
        assert metrics.rel_err_rows(a[:, sel], exact).max() <= 1e-5
    assert st["requests"] == 48 and st["p99_ms"] > 0
