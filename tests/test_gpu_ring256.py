"""The 256-transducer workload (ring of 110 mm, 512^2 grid at 0.45 mm, breast-like phantom,
720 rays per transducer, frequencies 100-800 kHz low to high, one per step) against the FP64
oracle's first frequency steps (stored by tests/golden/make_ring256_grid512.py, which calls
only the oracle): the plain FP32 form (tables of sampled transducers, predicted data,
gradient, direction, residual norm, image over the continuation) and the reduced-precision
forms, with the error of each result reported per frequency."""
import functools
import math
import os
import sys

import numpy as np
import pytest

import phantoms as ph
from oracle.medium import Grid, Ring, box_smooth, refractive_index
from oracle.step import StepSetup
from tests.gpu_cases import C0, abi_structs, oracle_tables_of, rel_l2, to_np

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "ring256_grid512_steps.npz")
W = ph.MEDIUM
IMAGE_GATE = 2e-3
PRECS = {"bf16": (2, 2.0 ** -9), "fp16": (3, 2.0 ** -12), "fp16x": (4, 2.0 ** -12)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def _gold():
    z = np.load(GOLD)
    return {k: z[k] for k in z.files}


@functools.lru_cache(maxsize=None)
def _setup():
    grid = Grid(W.nx, W.ny, W.dx, W.x0, W.y0, W.mask_radius)
    return StepSetup(grid, Ring(W.n_trans, W.radius, W.psi0), W.n_rays, W.ds, W.max_steps())


def _model(k):
    """The oracle's model at the start of step k (water for k = 0), float64 [ny][nx]."""
    st = _setup()
    c = np.full((st.grid.ny, st.grid.nx), C0)
    if k > 0:
        c.ravel()[st.grid.mask_index()] += _gold()["dc"][k - 1].astype(np.float64)
    return c


def _omega(k):
    return 2 * math.pi * float(_gold()["freqs_hz"][k])


D_OMEGA = 2 * math.pi * (W.freqs[1] - W.freqs[0])


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _abi_products(ctx, k, prec):
    """Predicted data and Q = 1 gradient of step k through the C ABI entry points."""
    import torch
    from paper_2211_00316_amd import _lib

    st = _setup()
    grid, ring, tp = abi_structs(st)
    win = int(_gold()["windows"][k])
    om = _omega(k)
    c = torch.as_tensor(_model(k), device="cuda:0")
    ns = ctx.refractive_index(grid, c, C0, win)
    tb = ctx.trace_rays(grid, ring, tp, ns)
    gr = ctx.build_green(tb, om, C0, prec=prec)
    q = torch.as_tensor(st.grid.mask_index(), device="cuda:0")
    cm = c.reshape(-1)[q]
    delta = (1.0 / cm ** 2 - (ns.reshape(-1)[q].double() / C0) ** 2).float()
    w = torch.full((q.numel(),), om * om * W.dx * W.dx, dtype=torch.complex64, device="cuda:0")
    d = ctx.born_forward(gr, w, delta)
    zero = torch.zeros(W.n_trans, W.n_trans, dtype=torch.complex64, device="cuda:0")
    pred = ctx.residual(tb, om, C0, zero, d)
    data = torch.as_tensor(_gold()["data"][k], device="cuda:0")
    R = ctx.residual(tb, om, C0, data, d)
    grad = ctx.born_adjoint(gr, w, R)
    return to_np(pred), to_np(grad)


def _step(ctx, k, prec, c_start=None):
    """One GPU step k from the oracle's model (or c_start); returns (c_new, dm, rn)."""
    import torch

    st = _setup()
    grid, ring, tp = abi_structs(st)
    c0 = _model(k) if c_start is None else c_start
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    rn = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    data = torch.as_tensor(_gold()["data"][k:k + 1], device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, int(_gold()["windows"][k]), [_omega(k)], [D_OMEGA],
                       data, float(_gold()["tau"]), residual_norm=rn, prec=prec)
    c_new = to_np(c_g)
    q = st.grid.mask_index()
    dm = (c_new.ravel()[q] ** -2 - c0.ravel()[q] ** -2) / float(_gold()["tau"])
    return c_new, dm, float(to_np(rn)[0])


def test_tables_of_sampled_transducers(ctx):
    # rays through the model after the first step (smoothed with the step's window): the
    # oracle traces 4 of the 256 transducers on the same FP32 map
    import torch

    st = _setup()
    grid, ring, tp = abi_structs(st)
    ns = box_smooth(refractive_index(_model(1), C0), int(_gold()["windows"][1]))
    ns32 = ns.astype(np.float32)
    _say("ring256 tables")
    tb = ctx.trace_rays(grid, ring, tp, torch.as_tensor(ns32, device="cuda:0"))
    emit = [0, 77, 130, 201]
    tb_o, _ = oracle_tables_of(st, ns32.astype(np.float64), emitters=emit)
    T, A, fl = to_np(tb.T)[emit], to_np(tb.A)[emit], to_np(tb.flags)[emit]
    v = ((fl & 0x80) != 0) & tb_o.valid
    mism = np.mean(((fl & 0x80) != 0) != tb_o.valid)
    eT, eA = rel_l2(T[v], tb_o.T[v]), rel_l2(A[v], tb_o.A[v])
    _say(f"  T {eT:.2e}  A {eA:.2e}  validity mismatch {mism:.2e}")
    assert eT <= 1e-5 and eA <= 1e-4 and mism <= 1e-4


@pytest.mark.parametrize("k", [0, 1, 2])
def test_fp32_step_products(ctx, k):
    from paper_2211_00316_amd import _lib

    g = _gold()
    _say(f"ring256 FP32 step {k}")
    pred, grad = _abi_products(ctx, k, _lib.RB_F32)
    _, dm, rn = _step(ctx, k, _lib.RB_F32)
    e = dict(data=rel_l2(pred, g["pred"][k]), grad=rel_l2(grad, g["grad"][k]),
             dm=rel_l2(dm, g["dm"][k]), rn=abs(rn - g["rn"][k]) / g["rn"][k])
    _say("  " + "  ".join(f"{n} {v:.2e}" for n, v in e.items()))
    assert max(e.values()) <= 1e-4


def _continuation(ctx, prec, steps):
    st = _setup()
    q = st.grid.mask_index()
    c = _model(0)
    out = []
    for k in range(steps):
        c, _, _ = _step(ctx, k, prec, c_start=c)
        ref = C0 + _gold()["dc"][k].astype(np.float64)
        out.append(float(np.linalg.norm(c.ravel()[q] - ref) / np.linalg.norm(ref - C0)))
    return out


def test_fp32_continuation_image(ctx):
    from paper_2211_00316_amd import _lib

    re = _continuation(ctx, _lib.RB_F32, len(_gold()["rn"]))
    _say("ring256 FP32 image RE per step " + " ".join(f"{x:.2e}" for x in re))
    assert max(re) <= 1e-4


@pytest.mark.parametrize("pname", list(PRECS))
def test_reduced_precision_per_frequency(ctx, pname):
    # 16-bit operands with per-transducer scales, FP32 accumulation, FP64 phase and update:
    # per frequency the error of the predicted data, the gradient and the direction against
    # the FP64 oracle, and the image over the continuation. The split FP16 form is held to the
    # image gate; the plain forms to 40 u.
    prec, u = PRECS[pname]
    g = _gold()
    K = len(g["rn"])
    rows = []
    for k in range(K):
        pred, grad = _abi_products(ctx, k, prec)
        _, dm, _ = _step(ctx, k, prec)
        rows.append((rel_l2(pred, g["pred"][k]), rel_l2(grad, g["grad"][k]),
                     rel_l2(dm, g["dm"][k])))
    re = _continuation(ctx, prec, K)
    for k in range(K):
        _say(f"ring256 {pname} f={g['freqs_hz'][k] / 1e3:.1f} kHz: data {rows[k][0]:.2e} "
             f"grad {rows[k][1]:.2e} dm {rows[k][2]:.2e} image RE {re[k]:.2e}")
    assert max(r[0] for r in rows) <= 40 * u and max(r[1] for r in rows) <= 40 * u
    if pname == "fp16x":
        assert max(r[2] for r in rows) <= IMAGE_GATE and max(re) <= IMAGE_GATE
    else:
        assert max(r[2] for r in rows) <= 40 * u and max(re) <= 40 * u
