"""Several frequency steps in one call (rb_frequency_sweep): against the FP64 oracle applied
step by step, against the same steps called one at a time, as a HIP graph replayed between
eager work, and its deferred error reports (conditions forced from the host)."""
import functools
import math
import sys

import numpy as np
import pytest

from oracle import step as ostep
from tests.gpu_cases import C0, abi_structs, case, rel_l2, to_np

pytestmark = pytest.mark.gpu

# Frequency continuation of two steps, low to high (Section 6.3.2): windows and sets.
WINDOWS = [3, 1]
SETS = [[2 * math.pi * 200e3], [2 * math.pi * 260e3, 2 * math.pi * 300e3]]


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _spacings(sets):
    out = []
    for s in sets:
        out.append([s[0]] if len(s) == 1 else [s[1] - s[0]] * len(s))
    return out


@functools.lru_cache(maxsize=None)
def _data(name):
    import phantoms as ph

    st, c_true = case(name)
    N = st.ring.n
    flat = [o for s in SETS for o in s]
    noise = ph.complex_noise((len(flat), N, N), 3)
    return ostep.synthesize(c_true, st, flat, noise, background="water")


def test_sweep_matches_oracle_steps(ctx):
    import torch

    st, _ = case("small")
    data = _data("small")
    c0 = np.full((st.grid.ny, st.grid.nx), C0)
    c_ref = c0.copy()
    f0 = 0
    for w, s, ds in zip(WINDOWS, SETS, _spacings(SETS)):
        c_ref = ostep.frequency_step(c_ref, st, s, ds, data[f0:f0 + len(s)], 0.12, window=w)
        f0 += len(s)
    grid, ring, tp = abi_structs(st)
    _say("frequency_sweep small, 2 steps")
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    ctx.frequency_sweep(grid, ring, tp, c_g, WINDOWS, SETS, _spacings(SETS),
                        torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12)
    q = st.grid.mask_index()
    dc = (to_np(c_g) - c0).ravel()[q]
    dc_ref = (c_ref - c0).ravel()[q]
    _say(f"  update rel L2 {rel_l2(dc, dc_ref):.2e}")
    assert rel_l2(dc, dc_ref) <= 2e-4


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16x"])
def test_sweep_and_graph_replays_equal_single_steps(ctx, pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"f32": _lib.RB_F32, "bf16": _lib.RB_BF16, "fp16x": _lib.RB_F16X}[pname]
    st, _ = case("small")
    grid, ring, tp = abi_structs(st)
    data = torch.as_tensor(_data("small").astype(np.complex64), device="cuda:0")
    c0 = torch.full((st.grid.ny, st.grid.nx), C0, dtype=torch.float64, device="cuda:0")
    # the steps one at a time
    c_ref = c0.clone()
    rn_ref = torch.zeros(len(SETS), dtype=torch.float64, device="cuda:0")
    f0 = 0
    for k, (w, s, ds) in enumerate(zip(WINDOWS, SETS, _spacings(SETS))):
        ctx.frequency_step(grid, ring, tp, c_ref, w, s, ds, data[f0:f0 + len(s)], 0.12,
                           residual_norm=rn_ref[k:k + 1], prec=prec)
        f0 += len(s)
    torch.cuda.synchronize()
    # one sweep without a graph
    c = c0.clone()
    rn = torch.zeros(len(SETS), dtype=torch.float64, device="cuda:0")
    ctx.frequency_sweep(grid, ring, tp, c, WINDOWS, SETS, _spacings(SETS), data, 0.12,
                        prec=prec, residual_norms=rn)
    assert torch.equal(c, c_ref)
    assert torch.allclose(rn, rn_ref, rtol=1e-12, atol=0)
    # captured once, then replayed; the program's own eager work and synchronisations in
    # between; every replay starts from the same model and must give the same result
    cg = c0.clone()
    rng = torch.zeros(len(SETS), dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        cg.copy_(c0)
        rng.zero_()
        ctx.frequency_sweep(grid, ring, tp, cg, WINDOWS, SETS, _spacings(SETS), data, 0.12,
                            prec=prec, use_graph=True, residual_norms=rng)
        torch.cuda.synchronize()
        _say(f"graph sweep {pname} replay {rep}")
        assert torch.equal(cg, c_ref), rep
        assert torch.allclose(rng, rn_ref, rtol=1e-12, atol=0), rep
        ns = ctx.refractive_index(grid, cg, C0, 3)       # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(ns).all()


def test_sweep_reports_non_finite_update(ctx):
    # A step length that drives m = c^-2 + tau dm negative: the first step fails, nothing is
    # committed, and the error names step 0.
    import torch
    from paper_2211_00316_amd import _lib

    st, _ = case("small")
    grid, ring, tp = abi_structs(st)
    data = torch.as_tensor(_data("small").astype(np.complex64), device="cuda:0")
    c0 = torch.full((st.grid.ny, st.grid.nx), C0, dtype=torch.float64, device="cuda:0")
    for use_graph in (False, True):
        c = c0.clone()
        with pytest.raises(_lib.RayBornError) as e:
            ctx.frequency_sweep(grid, ring, tp, c, WINDOWS, SETS, _spacings(SETS), data,
                                -1e30, use_graph=use_graph)
        assert e.value.status == _lib.RB_ENONFINITE
        assert "step 0" in str(e.value)
        assert torch.equal(c, c0)


def test_sweep_reports_ray_overflow(ctx):
    # max_steps too small for any ray to reach the ring: reported after the sweep, c kept.
    import torch
    from paper_2211_00316_amd import _lib

    st, _ = case("small")
    grid, ring, tp = abi_structs(st)
    short = _lib.TraceParams(tp.n_rays, 10, tp.ds, tp.c0)
    data = torch.as_tensor(_data("small").astype(np.complex64), device="cuda:0")
    c0 = torch.full((st.grid.ny, st.grid.nx), C0, dtype=torch.float64, device="cuda:0")
    c = c0.clone()
    with pytest.raises(_lib.RayBornError) as e:
        ctx.frequency_sweep(grid, ring, short, c, WINDOWS, SETS, _spacings(SETS), data, 0.12)
    assert e.value.status == _lib.RB_ENONFINITE
    assert "step 0" in str(e.value) and "max_steps" in str(e.value)
    assert torch.equal(c, c0)
