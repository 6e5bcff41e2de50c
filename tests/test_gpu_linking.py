"""Receiver tables by secant ray linking on the GPU (rb_set_receiver_linking) against the
FP64 oracle's linking (oracle.linking) on the same FP32-rounded map, the closed forms of
water (chords), a frequency step with linked receivers against the oracle's, and the
argument checks."""
import math
import sys

import numpy as np
import pytest

from oracle import linking, step as ostep
from oracle.medium import Grid
from tests.gpu_cases import C0, abi_structs, case, ns_of, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-8    # exit-angle tolerance of both sides (radians)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(max_iter=12):
    import torch
    from paper_2211_00316_amd import _lib

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = _lib.Context("cuda:0")
    ctx.set_receiver_linking(max_iter, TOL)
    return ctx


@pytest.mark.parametrize("name,window", [("small", 1), ("ragged", 5), ("ring64", 1)])
def test_linked_receiver_tables_match_oracle(name, window):
    import torch

    st, c = case(name)
    N = st.ring.n
    emitters = sorted({0, 1, N // 3, N // 2, N - 1})
    ns32 = np.asarray(ns_of(c, window), dtype=np.float32).astype(np.float64)
    _say(f"oracle linking {name} emitters {emitters}")
    lk = linking.link_receivers(ns32, st.grid, st.ring, st.n_rays, st.ds, st.max_steps,
                                emitters=emitters, tol=TOL)
    ctx = _ctx()
    grid, ring, tp = abi_structs(st)
    _say(f"GPU linking {name}")
    tb = ctx.trace_rays(grid, ring, tp, torch.as_tensor(ns32.astype(np.float32), device="cuda:0"))
    torch.cuda.synchronize()
    rows = torch.as_tensor(emitters, device="cuda:0")
    pick = lambda t: to_np(t.index_select(0, rows))
    valid = (pick(tb.rx_flags) & 0x80) != 0
    mism = int(np.count_nonzero(valid != lk.valid))
    both = valid & lk.valid
    eT = rel_l2(pick(tb.rx_T)[both], lk.T[both])
    eA = rel_l2(pick(tb.rx_A)[both], lk.A[both])
    _say(f"  valid mismatches {mism} of {valid.size}, rel L2 T {eT:.2e}, A {eA:.2e}")
    assert mism <= max(1, valid.size // 500)
    assert eT <= 1e-5 and eA <= 1e-4
    assert np.array_equal(pick(tb.rx_flags)[both] & 3, lk.K[both] & 3)
    ctx.close()


def test_linked_water_rays_are_chords():
    import torch

    st, _ = case("ring64")
    ctx = _ctx()
    grid, ring, tp = abi_structs(st)
    ns = torch.ones((st.grid.ny, st.grid.nx), dtype=torch.float32, device="cuda:0")
    tb = ctx.trace_rays(grid, ring, tp, ns)
    pos = st.ring.positions()
    chord = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    off = ~np.eye(st.ring.n, dtype=bool)
    valid = (to_np(tb.rx_flags) & 0x80) != 0
    assert valid[off].all() and not valid[~off].any()
    T = to_np(tb.rx_T)[off]
    A = to_np(tb.rx_A)[off].astype(np.float64)
    # The exit point lies within R TOL of the receiver; each step's length follows the
    # tracer's FP32 unit direction, whose norm is 1 to a few float ulps, and in water that
    # error has the same sign along the whole ray. Both stay far below 1e-6 of T (the
    # parity bar for travel times is 1e-5); a ray aimed or tallied wrongly is off by far more.
    eT = np.max(np.abs(T - chord[off] / C0) / (chord[off] / C0))
    eA = np.max(np.abs(A * np.sqrt(8 * math.pi * chord[off]) - 1.0))
    _say(f"water linking: max rel T error {eT:.2e}, max rel A error {eA:.2e}")
    assert eT <= 1e-6 and eA <= 1e-5
    ctx.close()


def test_frequency_step_with_linking_matches_oracle():
    import torch
    import phantoms as ph

    st, c_true = case("small")
    N = st.ring.n
    om = [2 * math.pi * 250e3]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((1, N, N), 2), background="water")
    # from a heterogeneous model the rays bend, so linked and interpolated receivers differ
    c0 = ostep.update(np.full_like(c_true, C0), (1.0 / c_true ** 2 - 1.0 / C0 ** 2).ravel()[
        st.grid.mask_index()], 0.5, st.grid)
    c_ref = ostep.frequency_step(c0, st, om, om, data, 0.12, link={"tol": TOL})
    c_fan = ostep.frequency_step(c0, st, om, om, data, 0.12)
    ctx = _ctx()
    grid, ring, tp = abi_structs(st)
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om,
                       torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12)
    q = st.grid.mask_index()
    dc = (to_np(c_g) - c0).ravel()[q]
    err = rel_l2(dc, (c_ref - c0).ravel()[q])
    sep = rel_l2((c_fan - c0).ravel()[q], (c_ref - c0).ravel()[q])
    _say(f"linked step: update rel L2 {err:.2e} (fan vs linked oracle steps differ by {sep:.2e})")
    assert err <= 1e-4 and sep > 5 * err
    ctx.close()


def test_linking_off_restores_interpolation_and_arguments_are_checked():
    import torch
    from paper_2211_00316_amd import _lib

    st, c = case("small")
    grid, ring, tp = abi_structs(st)
    ns = torch.as_tensor(np.asarray(ns_of(c, 1), dtype=np.float32), device="cuda:0")
    plain = _lib.Context("cuda:0")
    tb0 = plain.trace_rays(grid, ring, tp, ns)
    ctx = _ctx()
    ctx.set_receiver_linking(0, TOL)
    tb1 = ctx.trace_rays(grid, ring, tp, ns)
    torch.cuda.synchronize()
    assert torch.equal(tb0.rx_T, tb1.rx_T) and torch.equal(tb0.rx_flags, tb1.rx_flags)
    for bad in ((65, TOL), (-1, TOL), (4, 0.0), (4, 1e-3)):
        with pytest.raises(_lib.RayBornError) as e:
            ctx.set_receiver_linking(*bad)
        assert e.value.status == _lib.RB_EINVAL
    plain.close()
    ctx.close()
