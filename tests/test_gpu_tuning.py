"""Launch tuning and the fused multi-right-hand-side spreading, through the C ABI.

Every tuning changes only how the work is cut (tile edge, work-item size,
work-group shape, right-hand sides per work-group, FFT work-group width),
so every tuned plan must reproduce the FP64 oracle (O2) to the parity
tolerance and the default plan up to rounding order.
"""
import numpy as np
import pytest
import torch

from oracle import nfft as onfft, metrics, window
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL_O2 = {"f64": 1e-12, "f32": 1e-5}
# two launches of the same plan arithmetic in a different order
TOL_ORDER = {"f64": 1e-13, "f32": 2e-6}


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _plan(x, M, m, prec, max_rhs=1, tuning=None):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] N={x.shape[0]} d={x.shape[1]} M={M} m={m} {prec} rhs={max_rhs} tuning={tuning}",
          flush=True)
    return Plan(x, M, 2.0, m, precision=prec, max_rhs=max_rhs, device="cuda:0", tuning=tuning)


def _nodes(d, M, seed):
    """Uniform nodes plus grid-aligned nodes (closed edge) and a crowded
    cluster whose tile splits into several work items."""
    Ms = window.oversampled_size(M, 2.0)
    rng = np.random.default_rng(seed)
    return np.concatenate([wl.uniform_nodes(1500, d, seed),
                           rng.integers(-Ms // 2, Ms // 2, size=(200, d)) / Ms,
                           0.004 * rng.standard_normal((700, d))])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,M", [(1, 128), (2, 32)])
@pytest.mark.parametrize("nr,nrhs", [(2, 5), (4, 11), (8, 5), (8, 16)])
def test_fused_rhs_matches_oracle(d, M, nr, nrhs, prec):
    m = 5
    x = _nodes(d, M, 40 + d)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 41)) / N
    F = wl.complex_normal((nrhs, N), 42)
    p = _plan(x, M, m, prec, max_rhs=nrhs, tuning={"rhs_per_group": nr})
    assert p.tuning()["rhs_per_group"] == nr
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(F)))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(nrhs):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2[prec], r
    # the same plan with one right-hand side per work-group
    p.set_tuning("rhs_per_group", 1)
    sep = _np(p.adjoint(torch.from_numpy(F)))
    assert metrics.rel_err(got, sep) <= TOL_ORDER[prec]
    p.close()


TUNINGS = [
    {"tile_edge": 8},
    {"tile_edge": 32, "item_nodes": 64},
    {"item_nodes": 1024, "spread_threads": 64},
    {"spread_threads": 256, "fft_min_wg": 1},
    {"fft_min_wg": 65536},
    {"spread_planes": 2, "spread_mode": 1},
    {"tile_edge": 8, "spread_planes": 2, "spread_threads": 256, "spread_mode": 1},
    {"spread_mode": 2},
    {"spread_mode": 2, "tile_edge": 8, "item_nodes": 32},
    {"spread_mode": 2, "item_nodes": 1000},
    {"spread_mode": 2, "tile_edge": 32},   # padded edge 44 > 32: resolved to the LDS kernel
    {"spread_mode": 3},
    {"spread_mode": 3, "spread_planes": 2, "spread_threads": 64},
    {"spread_mode": 3, "tile_edge": 8, "item_nodes": 32, "spread_threads": 256},
    {"spread_mode": 3, "tile_edge": 32, "item_nodes": 1000},
    {"spread_mode": 4},
    {"spread_mode": 4, "spread_planes": 2, "spread_threads": 256},
    {"spread_mode": 4, "tile_edge": 8, "item_nodes": 32, "spread_threads": 64},
    {"spread_mode": 5},
    {"spread_mode": 5, "spread_threads": 256, "item_nodes": 1000},
    {"spread_mode": 5, "item_nodes": 32},
    {"spread_mode": 5, "item_nodes": 2048},
    {"spread_mode": 5, "tile_edge": 8},   # register tiles need tile edge 16: mode 4
    {"spread_mode": 5, "spread_threads": 512, "item_nodes": 1024},
    {"spread_mode": 6},
    {"spread_mode": 6, "item_nodes": 32},
    {"spread_mode": 6, "tile_edge": 8},   # the gather needs tile edge 16: mode 4
    {"spread_mode": 7},
    {"spread_mode": 7, "spread_threads": 256, "item_nodes": 1000},
    {"spread_mode": 7, "item_nodes": 32},
    {"spread_mode": 7, "item_nodes": 2048},
    {"spread_mode": 7, "tile_edge": 8},   # register tiles need tile edge 16: mode 4
    {"spread_mode": 7, "spread_threads": 512, "item_nodes": 1024},
    {"spread_mode": 7, "spread_threads": 64},
]

# the mode the register-tile kernels and the grid-tile gather resolve to where
# they do not apply (float64 for modes 5 and 6, a tile edge other than 16)
REG_FALLBACK = {5: 4, 6: 4, 7: 4}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("tuning", TUNINGS)
def test_tunings_agree(tuning, prec):
    M, m = 64, 6
    x = _nodes(2, M, 50)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 51)) / N
    f = wl.complex_normal(N, 52)
    fh = wl.complex_normal(M * M, 53)
    base = _plan(x, M, m, prec)
    base.set_weights(w)
    a0 = _np(base.adjoint(torch.from_numpy(f)))
    b0 = _np(base.forward(torch.from_numpy(fh)))
    p = _plan(x, M, m, prec, tuning=tuning)
    got_t = p.tuning()
    for k, v in tuning.items():
        if k == "spread_mode" and v == 2 and tuning.get("tile_edge") == 32:
            assert got_t[k] == 1
            continue
        # mode 7 at tile edge 16 in both precisions; modes 5 and 6 in float32
        reg = tuning.get("spread_mode") in REG_FALLBACK and tuning.get("tile_edge", 16) == 16 and \
            (prec == "f32" or tuning.get("spread_mode") == 7)
        if k == "spread_mode" and v in REG_FALLBACK and not reg:
            assert got_t[k] == REG_FALLBACK[v], got_t
            continue
        if k == "spread_threads" and v == 512 and not reg:
            assert got_t[k] == 256, got_t   # 512 threads: register tiles only
            continue
        assert got_t[k] == v, (k, got_t)
    p.set_weights(w)
    a = _np(p.adjoint(torch.from_numpy(f)))
    b = _np(p.forward(torch.from_numpy(fh)))
    assert metrics.rel_err(a, onfft.adjoint(x, w * f, M, 2.0, m)) <= TOL_O2[prec]
    assert metrics.rel_err(a, a0) <= TOL_ORDER[prec]
    assert metrics.rel_err(b, b0) <= TOL_ORDER[prec]
    base.close()
    p.close()


@pytest.mark.parametrize("prec,planes", [("f64", 1), ("f32", 1), ("f32", 2)])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 6, 7, 8])
def test_precomputed_window_factors(prec, planes, m):
    """Spread mode 3 reads the window factors from a table built once per node
    set with the same polynomials and arithmetic as the lanes of mode 1: the
    same plan switched between the two modes gives the same adjoint (float32
    single-rhs kernels sum in a fixed order, so up to the last bit there; the
    float64 kernels sum with LDS atomics), for one and for several
    right-hand sides; the forward's window sums use the table too once it
    exists; and the table costs 4 m reals per node."""
    M = 32
    x = _nodes(2, M, 90 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 91)) / N
    F = wl.complex_normal((3, N), 92)
    fh = wl.complex_normal((3, M * M), 93)
    p = _plan(x, M, m, prec, max_rhs=3, tuning={"spread_planes": planes} if prec == "f32" else None)
    p.set_weights(w)
    bytes0 = p.info()["bytes"]
    a1 = _np(p.adjoint(torch.from_numpy(F)))
    b1 = _np(p.forward(torch.from_numpy(fh)))
    p.set_tuning("spread_mode", 3)
    assert p.tuning()["spread_mode"] == 3
    rb = 8 if prec == "f64" else 4
    assert p.info()["bytes"] - bytes0 == N * 4 * m * rb
    a3 = _np(p.adjoint(torch.from_numpy(F)))
    tol = {"f64": 1e-14, "f32": 1e-7}[prec]
    for r in range(3):
        assert metrics.rel_err(a3[r], a1[r]) <= tol, r
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(3):
        assert metrics.rel_err(a3[r], ref[r]) <= TOL_O2[prec], r
    # the forward's window sums read the same table once it exists
    b3 = _np(p.forward(torch.from_numpy(fh)))
    for r in range(3):
        assert metrics.rel_err(b3[r], b1[r]) <= tol, r
        assert metrics.rel_err(b3[r], onfft.forward(x, fh[r], M, 2.0, m)) <= TOL_O2[prec], r
    # back to mode 1 and again to mode 3: the table is kept and reused
    p.set_tuning("spread_mode", 1)
    p.set_tuning("spread_mode", 3)
    assert p.info()["bytes"] - bytes0 == N * 4 * m * rb
    from paper_2302_00414_amd.nfft import nfft_footprint
    assert nfft_footprint(2, M, 2.0, m, N, prec, 3) >= p.info()["bytes"]
    assert metrics.rel_err(_np(p.adjoint(torch.from_numpy(F))), a3) <= tol
    p.close()


@pytest.mark.parametrize("prec,planes", [("f64", 1), ("f32", 1), ("f32", 2)])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 6, 8])
def test_window_evaluated_late(prec, planes, m):
    """Spread mode 4 evaluates the same window polynomials with the same
    arithmetic as mode 1, in another place of the pipeline: the same plan in
    the two modes gives the same adjoint (up to the last bit for the float32
    kernels, which sum in a fixed order), for one and for several right-hand
    sides, and needs no extra memory."""
    M = 32
    x = _nodes(2, M, 110 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 111)) / N
    F = wl.complex_normal((3, N), 112)
    p = _plan(x, M, m, prec, max_rhs=3, tuning={"spread_planes": planes} if prec == "f32" else None)
    p.set_weights(w)
    bytes0 = p.info()["bytes"]
    a1 = _np(p.adjoint(torch.from_numpy(F)))
    p.set_tuning("spread_mode", 4)
    assert p.tuning()["spread_mode"] == 4 and p.info()["bytes"] == bytes0
    a4 = _np(p.adjoint(torch.from_numpy(F)))
    tol = {"f64": 1e-14, "f32": 1e-7}[prec]
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(3):
        assert metrics.rel_err(a4[r], a1[r]) <= tol, r
        assert metrics.rel_err(a4[r], ref[r]) <= TOL_O2[prec], r
    p.close()


def test_set_tuning_rules():
    from paper_2302_00414_amd.nfft import NfftError
    x = wl.uniform_nodes(500, 2, 60)
    p = _plan(x, 32, 4, "f32")
    t = p.tuning()
    assert t == {"tile_edge": 16, "item_nodes": 256, "spread_threads": 128, "rhs_per_group": 1,
                 "fft_min_wg": 256, "spread_planes": 1, "spread_mode": 1}
    p.set_tuning("spread_threads", 64)
    assert p.tuning()["spread_threads"] == 64
    p.set_tuning("spread_threads", 0)          # back to the default
    assert p.tuning()["spread_threads"] == 128
    with pytest.raises(NfftError):
        p.set_tuning("tile_edge", 32)         # fixed at plan time
    with pytest.raises(NfftError):
        p.set_tuning("rhs_per_group", 3)
    assert p.tuning() == t
    p.close()


def test_3d_m8_float32():
    """d = 3 with m = 8 (float32 only: two float32 planes of 24^3 cells fit in LDS)."""
    x = _nodes(3, 16, 70)
    N = x.shape[0]
    w = np.full(N, 1.0 / N)
    f = wl.complex_normal(N, 71)
    p = _plan(x, 16, 8, "f32")
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    assert metrics.rel_err(got, onfft.adjoint(x, w * f, 16, 2.0, 8)) <= TOL_O2["f32"]
    fh = wl.complex_normal(16 ** 3, 72)
    assert metrics.rel_err(_np(p.forward(torch.from_numpy(fh))),
                           onfft.forward(x, fh, 16, 2.0, 8)) <= TOL_O2["f32"]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("min_wg", [1024, 65536])
def test_3d_merge_wide_first_stage(prec, min_wg):
    """d = 3, M = 32 (64-point lines, 4096 per pass), tile edge 8: with the FFT
    width tuning at 65536 work-groups every pass takes one line per
    work-group and a radix-2 first stage, so the merge loader sums the tile
    partials two elements a thread (at 1024, radix 8, eight a thread).
    Against the oracle (O2), adjoint and forward."""
    M, m = 32, 3
    x = _nodes(3, M, 75)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 76)) / N
    f = wl.complex_normal(N, 77)
    p = _plan(x, M, m, prec, tuning={"tile_edge": 8, "fft_min_wg": min_wg})
    assert p.tuning()["fft_min_wg"] == min_wg
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    assert metrics.rel_err(got, onfft.adjoint(x, w * f, M, 2.0, m)) <= TOL_O2[prec]
    fh = wl.complex_normal(M ** 3, 78)
    assert metrics.rel_err(_np(p.forward(torch.from_numpy(fh))),
                           onfft.forward(x, fh, M, 2.0, m)) <= TOL_O2[prec]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("m", [2, 6, 8])
@pytest.mark.parametrize("rpg", [1, 2])
def test_row_sweep_multi_rhs(prec, m, rpg):
    """Register row sweep with several right-hand sides in one launch, at the
    smallest and largest windows it covers (padded edge 16 + 2m <= 32)."""
    M, nrhs = 32, 3
    x = _nodes(2, M, 200 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 201)) / N
    F = wl.complex_normal((nrhs, N), 202)
    p = _plan(x, M, m, prec, max_rhs=nrhs, tuning={"spread_mode": 2, "rhs_per_group": rpg})
    assert p.tuning()["spread_mode"] == 2
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(F)))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(nrhs):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2[prec], r
    p.close()


@pytest.mark.parametrize("mode", [5, 7])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("items", [600, 1024])
@pytest.mark.parametrize("nt", [128, 256, 512])
def test_register_tile_spreading(mode, m, items, nt):
    """Spread modes 5 and 7 (float32, d = 2, tile edge 16) keep the padded
    tile of a work item in registers, on the vector ALUs (5) or as slots of
    matrix-core accumulators (7; 2m + 1 <= 16, so m = 8 resolves to 5):
    against the oracle (O2) and against the LDS kernel of mode 1 on the same
    plan (another summation order), for three right-hand sides, with
    grid-aligned nodes (closed edge), a crowded cluster whose tiles split
    into several work items, and work items longer than one staged batch of
    512 nodes."""
    M = 32
    x = _nodes(2, M, 300 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 301)) / N
    F = wl.complex_normal((3, N), 302)
    p = _plan(x, M, m, "f32", max_rhs=3, tuning={"item_nodes": items})
    p.set_weights(w)
    a1 = _np(p.adjoint(torch.from_numpy(F)))
    p.set_tuning("spread_mode", mode)
    p.set_tuning("spread_threads", nt)
    assert p.tuning()["spread_mode"] == (5 if mode == 7 and m == 8 else mode)
    got = _np(p.adjoint(torch.from_numpy(F)))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(3):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2["f32"], r
        assert metrics.rel_err(got[r], a1[r]) <= TOL_ORDER["f32"], r
    # fixed summation order: a second call gives the same bits
    again = _np(p.adjoint(torch.from_numpy(F)))
    assert np.array_equal(again, got)
    p.close()


@pytest.mark.parametrize("m", [1, 3, 6, 7])
@pytest.mark.parametrize("items", [600, 1024])
@pytest.mark.parametrize("nt", [128, 256])
def test_matrix_core_tile_float64(m, items, nt):
    """Spread mode 7 in float64 (v_mfma_f64_16x16x4f64, the accumulators and
    the sum of the waves' tiles in float64): against the oracle (O2) to the
    float64 parity tolerance, against the LDS kernel of mode 1 on the same
    plan (float64 LDS atomics, another order) to rounding, and two calls give
    the same bits (a fixed summation order, unlike the LDS atomics); three
    right-hand sides, grid-aligned nodes, crowded tiles, items of two
    batches."""
    M = 32
    x = _nodes(2, M, 500 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 501)) / N
    F = wl.complex_normal((3, N), 502)
    p = _plan(x, M, m, "f64", max_rhs=3, tuning={"item_nodes": items})
    p.set_weights(w)
    Ft = torch.from_numpy(F)
    a1 = _np(p.adjoint(Ft))
    p.set_tuning("spread_mode", 7)
    p.set_tuning("spread_threads", nt)
    assert p.tuning()["spread_mode"] == 7
    got = _np(p.adjoint(Ft))
    again = _np(p.adjoint(Ft))
    assert np.array_equal(got.view(np.uint64), again.view(np.uint64))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(3):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2["f64"], r
        assert metrics.rel_err(got[r], a1[r]) <= TOL_ORDER["f64"], r
    p.close()


@pytest.mark.parametrize("m", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("M,nrhs", [(32, 32), (32, 5), (64, 40), (16, 33)])
def test_grid_tile_gather(M, nrhs, m):
    """Spread mode 6 sums each grid cell of a 16 x 16 tile in one register
    for 32 right-hand sides at a time, visiting the nodes of the tile and of
    its eight neighbours (periodically: at M = 16 the grid has two tiles per
    dimension, so the neighbours on both sides are the same tile). Every
    right-hand side against the oracle (O2); against the register-tile
    kernel (mode 5) of the same plan up to rounding order; two calls give the
    same bits (one lane sums a cell in a fixed order). Right-hand-side counts
    below, at and above one group of 32; nodes uniform, on grid lines (closed
    edge) and crowded into one tile."""
    x = _nodes(2, M, 130 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 131)) / N
    F = wl.complex_normal((nrhs, N), 132 + nrhs)
    p = _plan(x, M, m, "f32", max_rhs=nrhs, tuning={"spread_mode": 6})
    assert p.tuning()["spread_mode"] == 6
    p.set_weights(w)
    Ft = torch.from_numpy(F)
    got = _np(p.adjoint(Ft))
    again = _np(p.adjoint(Ft))
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    e = metrics.rel_err_rows(got, ref)
    print(f"[gather] M={M} m={m} nrhs={nrhs}: max rel err vs O2 {e.max():.3e}", flush=True)
    assert e.max() <= TOL_O2["f32"]
    p.set_tuning("spread_mode", 5)
    reg = _np(p.adjoint(Ft))
    assert metrics.rel_err(got, reg) <= TOL_ORDER["f32"]
    p.close()


@pytest.mark.parametrize("m", [4, 6])
@pytest.mark.parametrize("items", [768, 1000])
def test_grid_tile_gather_long_units(items, m):
    """Spread mode 6 with units of several 128-entry staging rounds (768
    entries, the autotuner's choice on the spiral workload, and 1000, whose
    last round is partial): against the oracle (O2), against the register
    tile (mode 5) up to rounding order, and two calls give the same bits."""
    x = _nodes(2, 64, 140 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 141)) / N
    F = wl.complex_normal((40, N), 142)
    p = _plan(x, 64, m, "f32", max_rhs=40, tuning={"spread_mode": 6, "item_nodes": items})
    assert p.tuning()["spread_mode"] == 6 and p.tuning()["item_nodes"] == items
    p.set_weights(w)
    Ft = torch.from_numpy(F)
    got = _np(p.adjoint(Ft))
    again = _np(p.adjoint(Ft))
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    ref = onfft.adjoint(x, w[None, :] * F, 64, 2.0, m)
    e = metrics.rel_err_rows(got, ref)
    print(f"[gather] items={items} m={m}: max rel err vs O2 {e.max():.3e}", flush=True)
    assert e.max() <= TOL_O2["f32"]
    p.set_tuning("spread_mode", 5)
    reg = _np(p.adjoint(Ft))
    assert metrics.rel_err(got, reg) <= TOL_ORDER["f32"]
    p.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("items", [64, 256, 700])
def test_matrix_core_tiles_3d(m, items, prec):
    """Spread mode 7 for d = 3 (tile edge 8, 2m <= 8; m = 5 resolves to mode
    1): one wave holds the padded 3-D tile of its work item in matrix-core
    accumulators (float32 or float64). Against the oracle (O2) and against
    the LDS kernel of mode 1 on the same plan (another summation order), for
    three right-hand sides, with nodes on grid planes (closed edge), a
    crowded cluster whose tiles split into several work items, and work
    items longer than one staged batch of 256 nodes; two calls give the same
    bits."""
    M = 16
    x = _nodes(3, M, 400 + m)
    N = x.shape[0]
    w = (1.0 + 0.3 * wl.complex_normal(N, 401)) / N
    F = wl.complex_normal((3, N), 402)
    p = _plan(x, M, m, prec, max_rhs=3, tuning={"tile_edge": 8, "item_nodes": items})
    p.set_weights(w)
    Ft = torch.from_numpy(F)
    a1 = _np(p.adjoint(Ft))
    p.set_tuning("spread_mode", 7)
    assert p.tuning()["spread_mode"] == (1 if m == 5 else 7)
    got = _np(p.adjoint(Ft))
    again = _np(p.adjoint(Ft))
    u = np.uint32 if prec == "f32" else np.uint64
    if m != 5:
        assert np.array_equal(got.view(u), again.view(u))
    ref = onfft.adjoint(x, w[None, :] * F, M, 2.0, m)
    for r in range(3):
        assert metrics.rel_err(got[r], ref[r]) <= TOL_O2[prec], r
        assert metrics.rel_err(got[r], a1[r]) <= TOL_ORDER[prec], r
    p.close()
