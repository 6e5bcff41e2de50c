"""GPU-vs-oracle parity of every C-ABI entry point (HIP path on cuda:0, FP64 oracle on the
host, same seeded inputs). Tolerances (relative L2 over valid entries) follow the FP32 form:
travel time <= 1e-5, Green's functions, data and gradients <= 1e-4."""
import functools
import math
import sys

import numpy as np
import pytest

from oracle import born, green, step as ostep
from tests.gpu_cases import (C0, abi_structs, case, ns_of, oracle_tables, rel_l2,
                             tables_to_gpu, to_np)

pytestmark = pytest.mark.gpu

CASES = ["small", "ragged", "ring64"]


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("window", [1, 5])
def test_refractive_index(ctx, name, window):
    import torch

    st, c = case(name)
    grid, ring, tp = abi_structs(st)
    _say(f"refractive_index {name} w={window}")
    ns = ctx.refractive_index(grid, torch.as_tensor(c, device="cuda:0"), C0, window)
    ref = ns_of(c, window)
    assert np.max(np.abs(to_np(ns) - ref)) < 2e-7


@pytest.mark.parametrize("name", CASES)
def test_trace_rays_tables(ctx, name):
    import torch

    st, c = case(name)
    grid, ring, tp = abi_structs(st)
    tb_o, ns = oracle_tables(name)
    _say(f"trace_rays {name} N={st.ring.n} rays={st.n_rays} grid={st.grid.nx}")
    ns_g = torch.as_tensor(ns.astype(np.float32), device="cuda:0")
    tb = ctx.trace_rays(grid, ring, tp, ns_g)
    torch.cuda.synchronize()
    assert ctx.lost_nodes() == 0
    flags = to_np(tb.flags)
    valid = (flags & 0x80) != 0
    # the valid set is decided by geometry (coverage, 2 ds exclusion) on both sides
    mism = np.count_nonzero(valid != tb_o.valid)
    assert mism <= 1e-4 * valid.size, mism
    both = valid & tb_o.valid
    assert rel_l2(to_np(tb.T)[both], tb_o.T[both]) <= 1e-5
    assert rel_l2(to_np(tb.A)[both], tb_o.A[both]) <= 1e-4
    assert np.max(np.abs(to_np(tb.ux)[both] - tb_o.ux[both])) < 1e-4
    assert np.max(np.abs(to_np(tb.uy)[both] - tb_o.uy[both])) < 1e-4
    assert np.array_equal(flags[both] & 3, tb_o.K[both] & 3)
    rv = (to_np(tb.rx_flags) & 0x80) != 0
    assert np.array_equal(rv, tb_o.rx_valid)
    assert rel_l2(to_np(tb.rx_T)[rv], tb_o.rx_T[rv]) <= 1e-5
    assert rel_l2(to_np(tb.rx_A)[rv], tb_o.rx_A[rv]) <= 1e-4


def test_trace_rays_tables_folded_fans(ctx):
    # Triplicated region behind a slow lens: the general (smallest travel time) path.
    # Where two arrival sheets are closer than the FP32 rounding of the travel time, the
    # two sides may keep different sheets; those nodes are counted, not compared.
    import torch

    st, c = case("folded")
    grid, ring, tp = abi_structs(st)
    tb_o, ns = oracle_tables("folded")
    ns_g = torch.as_tensor(ns.astype(np.float32), device="cuda:0")
    _say("trace_rays folded")
    tb = ctx.trace_rays(grid, ring, tp, ns_g)
    torch.cuda.synchronize()
    valid = (to_np(tb.flags) & 0x80) != 0
    assert np.count_nonzero(valid != tb_o.valid) <= 1e-4 * valid.size
    both = valid & tb_o.valid
    T = to_np(tb.T)
    same = both & (np.abs(T - tb_o.T) <= 1e-6 * tb_o.T)
    other = np.count_nonzero(both & ~same)
    _say(f"  nodes on a different arrival sheet: {other} of {np.count_nonzero(both)}")
    assert other <= 1e-3 * np.count_nonzero(both)
    assert rel_l2(T[same], tb_o.T[same]) <= 1e-5
    # measured 4e-7 (FP32 fields; the caustic's largest amplitudes 2e-6)
    err_a = rel_l2(to_np(tb.A)[same], tb_o.A[same])
    _say(f"  amplitude rel. L2 on the same sheet: {err_a:.2e}")
    assert err_a <= 1e-5


def test_trace_rays_folded_fans_in_chunks_equal_one_launch():
    # A sample budget that splits the transducers into about five tracer chunks (the last one
    # ragged): every chunk's folded fans go through the rasterisation again, whose waves take
    # their runs from a counter reset per chunk, so the tables equal those of one launch
    # bitwise.
    import math
    import torch
    from paper_2211_00316_amd import _lib

    st, c = case("folded")
    grid, ring, tp = abi_structs(st)
    ns_g = torch.as_tensor(oracle_tables("folded")[1].astype(np.float32), device="cuda:0")
    n_mask = st.grid.mask_index().size
    per = (tp.max_steps + 1) * tp.n_rays * 25 + n_mask * 8 + tp.n_rays * 32
    out = []
    for budget in (1 << 30, per * math.ceil(st.ring.n / 5)):
        cx = _lib.Context("cuda:0")
        cx.set_sample_budget(budget)
        _say(f"trace_rays folded, sample budget {budget}")
        out.append(cx.trace_rays(grid, ring, tp, ns_g))
        torch.cuda.synchronize()
        cx.close()
    a, b = out
    for x, y in zip((a.T, a.A, a.ux, a.uy, a.flags, a.rx_T, a.rx_A, a.rx_flags),
                    (b.T, b.A, b.ux, b.uy, b.flags, b.rx_T, b.rx_A, b.rx_flags)):
        assert torch.equal(x, y)


def test_trace_rays_is_deterministic(ctx):
    import torch

    st, c = case("small")
    grid, ring, tp = abi_structs(st)
    ns = torch.as_tensor(oracle_tables("small")[1].astype(np.float32), device="cuda:0")
    a = ctx.trace_rays(grid, ring, tp, ns)
    b = ctx.trace_rays(grid, ring, tp, ns)
    torch.cuda.synchronize()
    for x, y in zip((a.T, a.A, a.ux, a.flags, a.rx_T), (b.T, b.A, b.ux, b.flags, b.rx_T)):
        assert torch.equal(x, y)


def test_trace_samples_count(ctx):
    # The tracer's unit of work: samples per ray are M + 1 (Definition 1 sampling, the source
    # sample included). A ray whose last full step lands within rounding of the ring may take
    # one step more or less on one side.
    import torch

    from oracle.trace import trace

    st, c = case("small")
    grid, ring, tp = abi_structs(st)
    ns = oracle_tables("small")[1]
    s = trace(ns, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, c0=st.c0)
    expect = int(np.sum(s.M[s.valid] + 1))
    ctx.trace_rays(grid, ring, tp, torch.as_tensor(ns.astype(np.float32), device="cuda:0"))
    torch.cuda.synchronize()
    got = ctx.trace_samples()
    _say(f"trace samples {got} (oracle {expect})")
    assert abs(got - expect) <= 2


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("f", [150e3, 800e3])
def test_build_green(ctx, name, f):
    st, c = case(name)
    tb_o, _ = oracle_tables(name)
    om = 2 * math.pi * f
    _say(f"build_green {name} f={f}")
    gr = ctx.build_green(tables_to_gpu(tb_o), om, C0)
    G, H, Hx, Hy = green.build_green(tb_o, om)
    assert rel_l2(to_np(gr.G), G) <= 1e-4
    assert rel_l2(to_np(gr.H[0]), H) <= 1e-4
    assert rel_l2(to_np(gr.H[1]), Hx) <= 1e-4
    assert rel_l2(to_np(gr.H[2]), Hy) <= 1e-4
    assert np.all(to_np(gr.G)[~tb_o.valid] == 0)


def _green_gpu(ctx, name, om):
    tb_o, _ = oracle_tables(name)
    G, H, Hx, Hy = green.build_green(tb_o, om)
    import torch
    from paper_2211_00316_amd import _lib

    gr = _lib.Green(torch.as_tensor(G.astype(np.complex64), device="cuda:0"),
                    torch.as_tensor(np.stack([H, Hx, Hy]).astype(np.complex64), device="cuda:0"))
    return tb_o, (G, H, Hx, Hy), gr


@pytest.mark.parametrize("name", CASES)
def test_born_forward(ctx, name):
    import torch

    st, c = case(name)
    om = 2 * math.pi * 300e3
    tb_o, (G, H, Hx, Hy), gr = _green_gpu(ctx, name, om)
    q = st.grid.mask_index()
    w = np.full(q.size, om ** 2 * st.grid.dx ** 2)
    delta = (1.0 / c.ravel()[q] ** 2 - 1.0 / C0 ** 2)
    _say(f"born_forward {name} N={st.ring.n} P_m={q.size}")
    d = ctx.born_forward(gr, torch.as_tensor(w.astype(np.complex64), device="cuda:0"),
                         torch.as_tensor(delta.astype(np.float32), device="cuda:0"))
    ref = born.forward(G, w, delta)
    assert rel_l2(to_np(d), ref) <= 1e-4
    dd = to_np(d)
    assert np.array_equal(dd, dd.T)  # reciprocity, exact by construction


@pytest.mark.parametrize("name", CASES)
def test_born_adjoint_and_dot_product(ctx, name):
    import torch

    st, c = case(name)
    om = 2 * math.pi * 400e3
    tb_o, (G, H, Hx, Hy), gr = _green_gpu(ctx, name, om)
    N, P = G.shape
    rng = np.random.default_rng(5)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    w = (om ** 2 * st.grid.dx ** 2) * np.exp(1j * rng.uniform(0, 0.3, P))
    _say(f"born_adjoint {name}")
    w_g = torch.as_tensor(w.astype(np.complex64), device="cuda:0")
    g = to_np(ctx.born_adjoint(gr, w_g, torch.as_tensor(R, device="cuda:0")))
    ref = born.adjoint(G, w.astype(np.complex64).astype(np.complex128), R.astype(np.complex128))
    assert rel_l2(g, ref) <= 1e-4
    # dot-product test on the GPU operators: <F delta, R> = <delta, F^H R>
    delta = rng.standard_normal(P).astype(np.float32)
    d = to_np(ctx.born_forward(gr, w_g, torch.as_tensor(delta, device="cuda:0")))
    lhs = np.real(np.vdot(d.astype(np.complex128), R.astype(np.complex128)))
    rhs = float(np.dot(delta.astype(np.float64), g.astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


@pytest.mark.parametrize("name", CASES)
def test_backproject(ctx, name):
    import torch

    st, c = case(name)
    om = 2 * math.pi * 350e3
    tb_o, (G, H, Hx, Hy), gr = _green_gpu(ctx, name, om)
    N, P = G.shape
    rng = np.random.default_rng(9)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    cq = c.ravel()[st.grid.mask_index()]
    _say(f"backproject {name}")
    dm = to_np(ctx.backproject(gr, torch.as_tensor(R, device="cuda:0"),
                               torch.as_tensor(cq, device="cuda:0"), om, 0.5 * om))
    S = born.backproject_weight(om, 0.5 * om, cq)
    ref = born.backproject(R.astype(np.complex128), H, Hx, Hy, S)
    assert rel_l2(dm, ref) <= 1e-4


@pytest.mark.parametrize("name", CASES)
def test_residual(ctx, name):
    import torch

    st, c = case(name)
    tb_o, _ = oracle_tables(name)
    N = st.ring.n
    om = 2 * math.pi * 600e3
    rng = np.random.default_rng(3)
    data = (1e-2 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))))
    dborn = (1e-3 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))))
    data = data.astype(np.complex64)
    dborn = dborn.astype(np.complex64)
    _say(f"residual {name}")
    R = to_np(ctx.residual(tables_to_gpu(tb_o), om, C0, torch.as_tensor(data, device="cuda:0"),
                           torch.as_tensor(dborn, device="cuda:0")))
    g = green.direct_data(tb_o, om)
    ref = ostep.residual(g + dborn, data, tb_o.rx_valid)
    assert rel_l2(R, ref) <= 1e-5
    assert np.all(R[~(tb_o.rx_valid & ~np.eye(N, dtype=bool))] == 0)


@pytest.mark.parametrize("name,window,mode", [("small", 1, 0), ("ring64", 1, 0),
                                              ("ragged", 5, 0), ("ragged", 5, 1)])
def test_frequency_step(ctx, name, window, mode):
    import torch
    import phantoms as ph

    st, c_true = case(name)
    N = st.ring.n
    freqs = [250e3] if name != "ragged" else [200e3, 260e3]
    om = [2 * math.pi * f for f in freqs]
    dom = [om[0]] if len(om) == 1 else [om[1] - om[0]] * len(om)
    noise = ph.complex_noise((len(om), N, N), 2)
    data = ostep.synthesize(c_true, st, om, noise, background="water")
    c0 = np.full_like(c_true, C0)
    oracle_mode = "ray_born" if mode == 0 else "ray_only"
    c_ref, parts = ostep.frequency_step(c0, st, om, dom, data, 0.12, window=window,
                                        mode=oracle_mode, return_parts=True)
    grid, ring, tp = abi_structs(st)
    _say(f"frequency_step {name} w={window} mode={mode}")
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    rn = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, window, om, dom,
                       torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12,
                       mode=mode, residual_norm=rn)
    c_new = to_np(c_g)
    q = st.grid.mask_index()
    dc_ref = (c_ref - c0).ravel()[q]
    dc = (c_new - c0).ravel()[q]
    assert rel_l2(dc, dc_ref) <= 1e-4, rel_l2(dc, dc_ref)
    outside = np.setdiff1d(np.arange(c0.size), q)
    assert np.all(c_new.ravel()[outside] == C0)
    rn_ref = sum(float(np.sum(np.abs(p["R"]) ** 2)) for p in parts["freqs"])
    assert abs(float(to_np(rn)[0]) - rn_ref) <= 1e-4 * rn_ref


def test_invalid_arguments_are_rejected(ctx):
    import torch
    from paper_2211_00316_amd import _lib

    st, c = case("small")
    grid, ring, tp = abi_structs(st)
    ns = torch.ones(st.grid.ny, st.grid.nx, dtype=torch.float32, device="cuda:0")
    bad = _lib.TraceParams(1, tp.max_steps, tp.ds, tp.c0)
    with pytest.raises(_lib.RayBornError) as e:
        ctx.trace_rays(grid, ring, bad, ns)
    assert e.value.status == _lib.RB_EINVAL
    big_ring = _lib.Ring(ring.n, 1.0, 0.0)
    with pytest.raises(_lib.RayBornError):
        ctx.trace_rays(grid, big_ring, tp, ns)
    with pytest.raises(_lib.RayBornError):
        ctx.refractive_index(grid, torch.as_tensor(c, device="cuda:0"), C0, 4)
    short = _lib.TraceParams(tp.n_rays, 10, tp.ds, tp.c0)
    with pytest.raises(_lib.RayBornError) as e:
        ctx.trace_rays(grid, ring, short, ns)
    assert e.value.status == _lib.RB_ENONFINITE
    # rows longer than 65535 nodes do not fit the 16-bit mask-run bounds of the binning
    wide = _lib.Grid(70000, 4, grid.dx, grid.x0, grid.y0, grid.mask_radius)
    ns_wide = torch.ones(4, 70000, dtype=torch.float32, device="cuda:0")
    with pytest.raises(_lib.RayBornError) as e:
        ctx.trace_rays(wide, ring, tp, ns_wide)
    assert e.value.status == _lib.RB_EINVAL


def test_nonfinite_update_leaves_model_unchanged(ctx):
    import torch

    st, c = case("small")
    N = st.ring.n
    grid, ring, tp = abi_structs(st)
    data = np.full((1, N, N), np.nan, dtype=np.complex64)
    c_g = torch.as_tensor(c.copy(), device="cuda:0")
    from paper_2211_00316_amd import _lib

    with pytest.raises(_lib.RayBornError) as e:
        ctx.frequency_step(grid, ring, tp, c_g, 1, [2 * math.pi * 2e5], [2 * math.pi * 2e5],
                           torch.as_tensor(data, device="cuda:0"), 0.12)
    assert e.value.status == _lib.RB_ENONFINITE
    assert np.array_equal(to_np(c_g), c)


# Reduced-precision form (16-bit operands, FP32 accumulation) -----------------------------
# Tolerances follow the unit roundoff u of the operand type (bf16 2^-9, fp16 2^-12 relative
# for round-to-nearest): operands <= 8u, contractions (two rounded factors, random-phase
# sums, a rounded epilogue factor) <= 40u. The image gate is relative to what the oracle's
# step changed, ||c_gpu - c_or|| / ||c_or - c_start|| over the mask, <= 2e-3: the split FP16
# form (fp16x) meets it; the plain forms do not (their rounding of H is amplified by the
# cancellation in the back-projection's double sum) and are held to 40u there.
LOWP = {"bf16": (2, 2.0 ** -9), "fp16": (3, 2.0 ** -12), "fp16x": (4, 2.0 ** -12)}
IMAGE_GATE = 2e-3


@pytest.mark.parametrize("pname", ["bf16", "fp16", "fp16x"])
@pytest.mark.parametrize("name,f", [("small", 500e3), ("ragged", 500e3), ("ring64", 500e3),
                                    ("ring64", 100e3), ("ring64", 1.2e6)])
def test_build_green_lowp(ctx, name, f, pname):
    # 16-bit operands with per-transducer power-of-two scales, at the lowest and highest
    # frequency of the continuation and in between: the unscaled values match the oracle, and
    # every stored row's largest value sits in [2^12, 2^14) for G (the bound from the row's
    # largest amplitude is tight) and below 2^14 for H.
    prec, u = LOWP[pname]
    st, c = case(name)
    tb_o, _ = oracle_tables(name)
    om = 2 * math.pi * f
    _say(f"build_green {pname} {name} {f:.0f} Hz")
    gr = ctx.build_green(tables_to_gpu(tb_o), om, C0, prec=prec)
    G, H, Hx, Hy = green.build_green(tb_o, om)
    errs = [rel_l2(to_np(gr.complex_G()), G)]
    Hs = to_np(gr.complex_H())
    errs += [rel_l2(Hs[k], ref) for k, ref in enumerate((H, Hx, Hy))]
    _say("  rel L2 G %.2e, H %.2e, Hx %.2e, Hy %.2e" % tuple(errs))
    assert max(errs) <= 8 * u
    sc = to_np(gr.scales).astype(np.float64)
    assert np.all(sc > 0) and np.array_equal(np.exp2(np.round(np.log2(sc))), sc)
    Gs = np.abs(to_np(gr.G.float()))[:, :, :G.shape[1]].max(axis=(0, 2))
    rows = tb_o.valid.any(axis=1)
    assert np.all(Gs < 2.0 ** 14) and np.all(Gs[rows] >= 2.0 ** 12)
    assert np.abs(to_np(gr.H.float())).max() < 2.0 ** 14
    if pname == "fp16x":
        # the high and low parts together carry H to about u^2
        assert max(errs[1:]) <= 4 * u * u + 1e-6


def _green_gpu_lowp(ctx, name, om, prec):
    tb_o, _ = oracle_tables(name)
    return tb_o, green.build_green(tb_o, om), ctx.build_green(tables_to_gpu(tb_o), om, C0,
                                                             prec=prec)


@pytest.mark.parametrize("pname", ["bf16", "fp16"])
@pytest.mark.parametrize("name", ["small", "ragged", "ring64"])
def test_born_forward_lowp(ctx, name, pname):
    import torch

    prec, u = LOWP[pname]
    st, c = case(name)
    om = 2 * math.pi * 300e3
    tb_o, (G, H, Hx, Hy), gr = _green_gpu_lowp(ctx, name, om, prec)
    q = st.grid.mask_index()
    w = np.full(q.size, om ** 2 * st.grid.dx ** 2)
    delta = (1.0 / c.ravel()[q] ** 2 - 1.0 / C0 ** 2)
    _say(f"born_forward {pname} {name}")
    d = to_np(ctx.born_forward(gr, torch.as_tensor(w.astype(np.complex64), device="cuda:0"),
                               torch.as_tensor(delta.astype(np.float32), device="cuda:0")))
    ref = born.forward(G, w, delta)
    err = rel_l2(d, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 40 * u
    assert np.array_equal(d, d.T)


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16"])
@pytest.mark.parametrize("n,n_mask", [(64, 37), (300, 1000), (1024, 4133)])
def test_born_forward_carried_weights(ctx, n, n_mask, pname):
    # Operands that already carry sqrt(v) (w = delta = NULL), as inside a frequency step:
    # d = G G^T. Seeded G rounded to the operand type on the host; the oracle takes the
    # rounded values, so only the FP32 accumulation differs. Shapes: one tile; several
    # 256 x 128 tiles with a ragged last row and column block and a ragged node count (zeros
    # past n_mask); the ring size of the large workload.
    import torch
    from paper_2211_00316_amd import _lib

    rng = np.random.default_rng(n * 7919 + n_mask)
    G = rng.standard_normal((n, n_mask)) + 1j * rng.standard_normal((n, n_mask))
    if pname == "f32":
        prec = _lib.RB_F32
        Gq = G.astype(np.complex64)
        gr = _lib.Green.empty(n, n_mask, "cuda:0", prec)
        gr.G.copy_(torch.as_tensor(Gq))
        Gq = Gq.astype(np.complex128)
    else:
        prec = LOWP[pname][0]
        dt = torch.bfloat16 if pname == "bf16" else torch.float16
        re = torch.as_tensor(G.real).to(dt)
        im = torch.as_tensor(G.imag).to(dt)
        Gq = re.double().numpy() + 1j * im.double().numpy()
        gr = _lib.Green.empty(n, n_mask, "cuda:0", prec)
        gr.G.zero_()
        gr.G[0, :, :n_mask].copy_(re)
        gr.G[1, :, :n_mask].copy_(im)
    _say(f"born_forward carried weights {pname} n={n} n_mask={n_mask}")
    d = to_np(ctx.born_forward(gr, None, None))
    ref = born.forward(Gq, np.ones(n_mask), np.ones(n_mask))
    err = rel_l2(d, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 1e-5
    assert np.array_equal(d, d.T)


@pytest.mark.parametrize("pname", ["bf16", "fp16", "fp16x"])
@pytest.mark.parametrize("name", ["small", "ragged", "ring64"])
def test_backproject_lowp(ctx, name, pname):
    import torch

    prec, u = LOWP[pname]
    st, c = case(name)
    om = 2 * math.pi * 350e3
    tb_o, (G, H, Hx, Hy), gr = _green_gpu_lowp(ctx, name, om, prec)
    N = G.shape[0]
    rng = np.random.default_rng(9)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    cq = c.ravel()[st.grid.mask_index()]
    _say(f"backproject {pname} {name}")
    dm = to_np(ctx.backproject(gr, torch.as_tensor(R, device="cuda:0"),
                               torch.as_tensor(cq, device="cuda:0"), om, 0.5 * om))
    S = born.backproject_weight(om, 0.5 * om, cq)
    ref = born.backproject(R.astype(np.complex128), H, Hx, Hy, S)
    err = rel_l2(dm, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= (4 * u if pname == "fp16x" else 40 * u)


@pytest.mark.parametrize("pname", ["bf16", "fp16", "fp16x"])
@pytest.mark.parametrize("name,window", [("ring64", 1), ("ragged", 5)])
def test_frequency_step_lowp_image(ctx, name, window, pname):
    import torch
    import phantoms as ph

    prec, u = LOWP[pname]
    st, c_true = case(name)
    N = st.ring.n
    om = [2 * math.pi * 250e3]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((1, N, N), 2), background="water")
    c0 = np.full_like(c_true, C0)
    c_ref = ostep.frequency_step(c0, st, om, om, data, 0.12, window=window)
    grid, ring, tp = abi_structs(st)
    _say(f"frequency_step {pname} {name} w={window}")
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, window, om, om,
                       torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12,
                       prec=prec)
    q = st.grid.mask_index()
    c_new = to_np(c_g).ravel()[q]
    img = rel_l2(c_new, c_ref.ravel()[q])   # ||c||-normalised (printed only)
    re = float(np.linalg.norm(c_new - c_ref.ravel()[q]) /
               np.linalg.norm((c_ref - c0).ravel()[q]))   # the gate: relative to the change
    _say(f"  image RE {re:.2e} (||c||-normalised {img:.2e})")
    assert re <= (IMAGE_GATE if pname == "fp16x" else 40 * u)


@functools.lru_cache(maxsize=None)
def _wide_reference(window):
    """Oracle step of the "wide" case from water (data, start and result)."""
    import phantoms as ph

    st, c_true = case("wide")
    N = st.ring.n
    om = [2 * math.pi * 250e3]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((1, N, N), 2), background="water")
    c0 = np.full_like(c_true, C0)
    return om, data, c0, ostep.frequency_step(c0, st, om, om, data, 0.12, window=window)


@pytest.mark.parametrize("pname", ["bf16", "fp16x"])
def test_frequency_step_lowp_image_wide(ctx, pname):
    """The step's 16-bit operands over several row slabs and a partial last block of 64
    transducers (the split form's FP8 low parts are stored in such blocks), against the
    oracle with the image gate of the reduced-precision form."""
    import torch

    prec, u = LOWP[pname]
    st, _ = case("wide")
    om, data, c0, c_ref = _wide_reference(5)
    grid, ring, tp = abi_structs(st)
    _say(f"frequency_step {pname} wide (N = {st.ring.n}) w=5")
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, 5, om, om,
                       torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12,
                       prec=prec)
    q = st.grid.mask_index()
    c_new = to_np(c_g).ravel()[q]
    re = float(np.linalg.norm(c_new - c_ref.ravel()[q]) /
               np.linalg.norm((c_ref - c0).ravel()[q]))
    _say(f"  image RE {re:.2e}")
    assert re <= (IMAGE_GATE if pname == "fp16x" else 40 * u)
