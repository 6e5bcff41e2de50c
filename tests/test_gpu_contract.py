"""The boundary's workspace and asynchrony contract (C ABI, HIP path on cuda:0):
rb_reserve sizes every workspace up front, after which a frequency step allocates nothing;
a step with a device report needs no host synchronisation and can be captured into a HIP
graph by the caller, one step at a time; the 16-bit adjoint matches the oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import born, step as ostep
from tests.gpu_cases import C0, abi_structs, case, oracle_tables, rel_l2, tables_to_gpu, to_np

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _step_inputs(name="ring64", freqs=(250e3,)):
    import phantoms as ph

    st, c_true = case(name)
    N = st.ring.n
    om = [2 * math.pi * f for f in freqs]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((len(om), N, N), 2),
                            background="water")
    return st, c_true, om, data


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16x"])
def test_reserved_context_steps_without_allocating(pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"f32": _lib.RB_F32, "bf16": _lib.RB_BF16, "fp16x": _lib.RB_F16X}[pname]
    st, c_true, om, data = _step_inputs()
    grid, ring, tp = abi_structs(st)
    ctx = _lib.Context("cuda:0")
    budget = 1 << 30
    ctx.set_sample_budget(budget)
    _say(f"reserve {pname}")
    ctx.reserve(grid, ring, tp, prec)
    c0 = np.full_like(c_true, C0)
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    d_g = torch.as_tensor(data.astype(np.complex64), device="cuda:0")
    rep = torch.zeros(_lib.REPORT_BYTES, dtype=torch.uint8, device="cuda:0")
    # first step: the library's code object is loaded by the first launches
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om, d_g, 0.12, prec=prec)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om, d_g, 0.12, prec=prec)
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om, d_g, 0.12, prec=prec, report=rep)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _say(f"  free before {free0}, after {free1}")
    assert free1 == free0
    r = _lib.decode_report(rep)
    assert r.status == _lib.RB_OK and r.flags == 0 and r.lost_nodes == 0
    assert r.ray_samples > st.ring.n * st.n_rays
    # the reservation covers exactly what rb_workspace_bytes names for the geometry
    assert _lib.workspace_bytes(grid, ring, tp, prec, budget) > 0
    # a call beyond the reservation fails before launching anything
    more = _lib.TraceParams(tp.n_rays * 2, tp.max_steps, tp.ds, tp.c0)
    c_keep = to_np(c_g).copy()
    with pytest.raises(_lib.RayBornError) as e:
        ctx.frequency_step(grid, ring, more, c_g, 1, om, om, d_g, 0.12, prec=prec)
    assert e.value.status == _lib.RB_ENOMEM
    other = _lib.Grid(grid.nx, grid.ny, grid.dx, grid.x0, grid.y0, grid.mask_radius * 0.9)
    with pytest.raises(_lib.RayBornError) as e:
        ctx.frequency_step(other, ring, tp, c_g, 1, om, om, d_g, 0.12, prec=prec)
    assert e.value.status == _lib.RB_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(to_np(c_g), c_keep)
    assert torch.cuda.mem_get_info()[0] == free1
    ctx.close()


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16x"])
def test_single_step_captured_by_the_caller(pname):
    # One rb_frequency_step with a device report, captured into the caller's HIP graph on the
    # context's stream and replayed several times with eager work and synchronisations in
    # between: every replay equals the eager step bitwise.
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"f32": _lib.RB_F32, "bf16": _lib.RB_BF16, "fp16x": _lib.RB_F16X}[pname]
    st, c_true, om, data = _step_inputs("ragged", (200e3, 260e3))
    dom = [om[1] - om[0]] * 2
    grid, ring, tp = abi_structs(st)
    s = torch.cuda.Stream()
    ctx = _lib.Context("cuda:0", stream=s)
    ctx.set_sample_budget(1 << 30)
    ctx.reserve(grid, ring, tp, prec)
    c_start = torch.as_tensor(np.full_like(c_true, C0), device="cuda:0")
    d_g = torch.as_tensor(data.astype(np.complex64), device="cuda:0")
    c_g = c_start.clone()
    rn = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    rep = torch.zeros(_lib.REPORT_BYTES, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        ctx.frequency_step(grid, ring, tp, c_g, 5, om, dom, d_g, 0.12, residual_norm=rn,
                           prec=prec, report=rep)
    torch.cuda.synchronize()
    c_eager = c_g.clone()
    rn_eager = rn.clone()
    assert _lib.decode_report(rep).status == _lib.RB_OK
    _say(f"capture {pname}")
    c_g.copy_(c_start)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        ctx.frequency_step(grid, ring, tp, c_g, 5, om, dom, d_g, 0.12, residual_norm=rn,
                           prec=prec, report=rep)
    torch.cuda.synchronize()
    for k in range(3):
        c_g.copy_(c_start)
        rn.zero_()
        rep.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _say(f"  replay {k}")
        assert torch.equal(c_g, c_eager)
        # the residual norm adds per-workgroup sums with atomics: equal up to their order
        assert torch.allclose(rn, rn_eager, rtol=1e-12, atol=0)
        assert _lib.decode_report(rep).status == _lib.RB_OK
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda:0")
        assert float((x * 0).abs().sum()) == 0.0
    del g
    ctx.close()


def test_report_of_a_rejected_step():
    import torch
    from paper_2211_00316_amd import _lib

    st, c = case("small")
    N = st.ring.n
    grid, ring, tp = abi_structs(st)
    ctx = _lib.Context("cuda:0")
    data = torch.full((1, N, N), float("nan"), dtype=torch.complex64, device="cuda:0")
    c_g = torch.as_tensor(c.copy(), device="cuda:0")
    rep = torch.zeros(_lib.REPORT_BYTES, dtype=torch.uint8, device="cuda:0")
    om = [2 * math.pi * 2e5]
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om, data, 0.12, report=rep)  # no raise
    torch.cuda.synchronize()
    r = _lib.decode_report(rep)
    assert r.status == _lib.RB_ENONFINITE and (r.flags & 2)
    assert np.array_equal(to_np(c_g), c)
    ctx.close()


@pytest.mark.parametrize("pname,u", [("bf16", 2.0 ** -9), ("fp16", 2.0 ** -12)])
@pytest.mark.parametrize("name", ["small", "ragged", "ring64"])
def test_born_adjoint_lowp(name, pname, u):
    # Eq. functional-gradient (Q = 1) with 16-bit operands: the oracle's adjoint on the same
    # tables, and the dot-product test against the 16-bit forward.
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"bf16": _lib.RB_BF16, "fp16": _lib.RB_F16}[pname]
    st, c = case(name)
    om = 2 * math.pi * 400e3
    tb_o, _ = oracle_tables(name)
    from oracle import green

    G = green.build_green(tb_o, om)[0]
    ctx = _lib.Context("cuda:0")
    gr = ctx.build_green(tables_to_gpu(tb_o), om, C0, prec=prec)
    N, P = G.shape
    rng = np.random.default_rng(5)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    w = (om ** 2 * st.grid.dx ** 2) * np.exp(1j * rng.uniform(0, 0.3, P))
    w_g = torch.as_tensor(w.astype(np.complex64), device="cuda:0")
    _say(f"born_adjoint {pname} {name}")
    g = to_np(ctx.born_adjoint(gr, w_g, torch.as_tensor(R, device="cuda:0")))
    ref = born.adjoint(G, w.astype(np.complex64).astype(np.complex128), R.astype(np.complex128))
    err = rel_l2(g, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 40 * u
    delta = rng.standard_normal(P).astype(np.float32)
    d = to_np(ctx.born_forward(gr, w_g, torch.as_tensor(delta, device="cuda:0")))
    lhs = np.real(np.vdot(d.astype(np.complex128), R.astype(np.complex128)))
    rhs = float(np.dot(delta.astype(np.float64), g.astype(np.float64)))
    assert abs(lhs - rhs) <= 40 * u * abs(lhs)
    ctx.close()
