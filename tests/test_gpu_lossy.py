"""GPU-vs-oracle parity of the absorbing, dispersive path (Szabo's model: Section 2.2, Eqs.
szabo_dispersion_equation, wave-number, amplitude-abs-discretised, scattering-potential, and
Section 3.4's d|kbar|/domega): rb_lossy_maps, rb_trace_rays_lossy, rb_backproject_lossy and
rb_frequency_step_lossy in every operand form, against the FP64 oracle (oracle.lossy and the
absorption arguments of oracle.step) on the same seeded inputs. Tolerances as for the lossless
entry points: maps to FP32 rounding, travel time <= 1e-5 and amplitudes <= 1e-4 (relative L2),
FP32 steps <= 1e-4, 16-bit images at the lossless gates."""
import dataclasses
import functools
import math
import sys

import numpy as np
import pytest

from oracle import born, green, linking, lossy, step as ostep
from oracle.medium import box_smooth
from tests.gpu_cases import (C0, abi_structs, absorption_case, case, ns_of, rel_l2,
                             tables_to_gpu, to_np)

pytestmark = pytest.mark.gpu

Y = 1.4
CASES = ["small", "ragged", "ring64"]
LOWP = {"bf16": (2, 2.0 ** -9), "fp16": (3, 2.0 ** -12), "fp16x": (4, 2.0 ** -12)}
IMAGE_GATE = 2e-3


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _maps32(name, om, window):
    """The oracle's maps of omega rounded to FP32 (the tracer's input) and box_w(alpha0)."""
    st, c = case(name)
    al = box_smooth(absorption_case(name, Y), window)
    n_w = lossy.tracing_index(ns_of(c, window), al, om, Y, C0)
    return n_w.astype(np.float32), (om ** Y * al).astype(np.float32), al


WORKERS = 8   # oracle processes for the tables (the GPU tests run in one process)


@functools.lru_cache(maxsize=None)
def _lossy_oracle_tables(name, om, window=1):
    """Oracle tables of the FP32-rounded map of omega (the tracer's input), with B."""
    st, c = case(name)
    n32, a32, _ = _maps32(name, om, window)
    ab = lossy.Absorption(absorption_case(name, Y), Y)
    tb, _ = ostep.tables_for(c, st, window, map32=True, absorption=ab, omega=om,
                             workers=WORKERS)
    return tb, n32, a32


def _with_absorption(tb, om):
    """Tables whose amplitudes include A_abs (the form the GPU tables take)."""
    return dataclasses.replace(tb, A=tb.A * lossy.absorption_factor(om, tb.B, Y),
                               rx_A=tb.rx_A * lossy.absorption_factor(om, tb.rx_B, Y),
                               B=None, rx_B=None)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("window", [1, 5])
def test_lossy_maps(ctx, name, window):
    st, c = case(name)
    a = absorption_case(name, Y)
    grid, ring, tp = abi_structs(st)
    om = 2 * math.pi * 500e3
    _say(f"lossy_maps {name} w={window}")
    n_w, a_w = ctx.lossy_maps(grid, _dev(c), _dev(a), Y, C0, om, window)
    al = box_smooth(a, window)
    ref_n = lossy.tracing_index(ns_of(c, window), al, om, Y, C0)
    assert np.max(np.abs(to_np(n_w) - ref_n)) < 2e-7
    ref_a = om ** Y * al
    assert np.max(np.abs(to_np(a_w) - ref_a)) <= 1e-6 * np.max(ref_a)
    # dispersion is present: the map differs from the lossless index where alpha0 > 0
    assert np.max(np.abs(ref_n - ns_of(c, window))) > 1e-4
    # alpha0 = 0: the lossless index to the bit, and no absorption
    z0, za = ctx.lossy_maps(grid, _dev(c), _dev(np.zeros_like(a)), Y, C0, om, window)
    ns = ctx.refractive_index(grid, _dev(c), C0, window)
    assert np.array_equal(to_np(z0), to_np(ns)) and np.all(to_np(za) == 0)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("f", [200e3, 900e3])
def test_trace_rays_lossy_tables(ctx, name, f):
    import torch

    st, c = case(name)
    om = 2 * math.pi * f
    grid, ring, tp = abi_structs(st)
    tb_o, n32, a32 = _lossy_oracle_tables(name, om)
    ref = _with_absorption(tb_o, om)
    _say(f"trace_rays_lossy {name} f={f}")
    tb = ctx.trace_rays_lossy(grid, ring, tp, _dev(n32), _dev(a32))
    torch.cuda.synchronize()
    assert ctx.lost_nodes() == 0
    flags = to_np(tb.flags)
    valid = (flags & 0x80) != 0
    assert np.count_nonzero(valid != ref.valid) <= 1e-4 * valid.size
    both = valid & ref.valid
    assert rel_l2(to_np(tb.T)[both], ref.T[both]) <= 1e-5
    eA = rel_l2(to_np(tb.A)[both], ref.A[both])
    _say(f"  rel L2 A {eA:.2e}; absorption at the far side {np.min(ref.A[both] / tb_o.A[both]):.3f}")
    assert eA <= 1e-4
    assert np.array_equal(flags[both] & 3, ref.K[both] & 3)
    rv = (to_np(tb.rx_flags) & 0x80) != 0
    assert np.array_equal(rv, ref.rx_valid)
    assert rel_l2(to_np(tb.rx_T)[rv], ref.rx_T[rv]) <= 1e-5
    assert rel_l2(to_np(tb.rx_A)[rv], ref.rx_A[rv]) <= 1e-4


def test_linked_receivers_lossy(ctx):
    import torch
    from paper_2211_00316_amd import _lib

    name = "small"
    st, c = case(name)
    om = 2 * math.pi * 700e3
    N = st.ring.n
    emitters = [0, N // 3, N - 1]
    n32, a32, al = _maps32(name, om, 1)
    _say("oracle linking, lossy")
    lk = linking.link_receivers(n32.astype(np.float64), st.grid, st.ring, st.n_rays, st.ds,
                                st.max_steps, emitters=emitters, tol=1e-8, alpha=al)
    lctx = _lib.Context("cuda:0")
    lctx.set_receiver_linking(12, 1e-8)
    grid, ring, tp = abi_structs(st)
    _say("GPU linking, lossy")
    tb = lctx.trace_rays_lossy(grid, ring, tp, _dev(n32), _dev(a32))
    torch.cuda.synchronize()
    rows = torch.as_tensor(emitters, device="cuda:0")
    pick = lambda t: to_np(t.index_select(0, rows))
    valid = (pick(tb.rx_flags) & 0x80) != 0
    both = valid & lk.valid
    assert np.count_nonzero(valid != lk.valid) <= max(1, valid.size // 500)
    A_ref = lk.A * lossy.absorption_factor(om, lk.B, Y)
    assert rel_l2(pick(tb.rx_T)[both], lk.T[both]) <= 1e-5
    assert rel_l2(pick(tb.rx_A)[both], A_ref[both]) <= 1e-4


def _operands(name, om):
    st, c = case(name)
    tb_o, _, _ = _lossy_oracle_tables(name, om)
    G, H, Hx, Hy = green.build_green(tb_o, om, C0, Y)
    return st, c, tb_o, (G, H, Hx, Hy)


@pytest.mark.parametrize("name", CASES)
def test_backproject_lossy(ctx, name):
    import torch
    from paper_2211_00316_amd import _lib

    om = 2 * math.pi * 350e3
    st, c, tb_o, (G, H, Hx, Hy) = _operands(name, om)
    gr = _lib.Green(_dev(G.astype(np.complex64)),
                    _dev(np.stack([H, Hx, Hy]).astype(np.complex64)))
    N = G.shape[0]
    rng = np.random.default_rng(9)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    q = st.grid.mask_index()
    cq = c.ravel()[q]
    aq = absorption_case(name, Y).ravel()[q]
    _say(f"backproject_lossy {name}")
    dm = to_np(ctx.backproject_lossy(gr, _dev(R), _dev(cq), _dev(aq), Y, om, 0.5 * om))
    S = born.backproject_weight(om, 0.5 * om, cq, aq, Y)
    ref = born.backproject(R.astype(np.complex128), H, Hx, Hy, S)
    err = rel_l2(dm, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 1e-4
    # the imaginary part of S (about 2e-3 of S in the absorbing blob) is resolved: without it
    # the direction moves by more than the GPU's distance to the oracle
    ref_re = born.backproject(R.astype(np.complex128), H, Hx, Hy, S.real)
    assert rel_l2(ref_re, ref) > 2e-4
    assert err < 0.5 * rel_l2(dm, ref_re)
    torch.cuda.synchronize()


@pytest.mark.parametrize("pname", ["bf16", "fp16", "fp16x"])
def test_backproject_lossy_lowp(ctx, pname):
    prec, u = LOWP[pname]
    name = "ring64"
    om = 2 * math.pi * 350e3
    st, c, tb_o, (G, H, Hx, Hy) = _operands(name, om)
    gr = ctx.build_green(tables_to_gpu(_with_absorption(tb_o, om)), om, C0, prec=prec)
    N = G.shape[0]
    rng = np.random.default_rng(9)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    q = st.grid.mask_index()
    cq = c.ravel()[q]
    aq = absorption_case(name, Y).ravel()[q]
    _say(f"backproject_lossy {pname} {name}")
    dm = to_np(ctx.backproject_lossy(gr, _dev(R), _dev(cq), _dev(aq), Y, om, 0.5 * om))
    S = born.backproject_weight(om, 0.5 * om, cq, aq, Y)
    ref = born.backproject(R.astype(np.complex128), H, Hx, Hy, S)
    err = rel_l2(dm, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= (4 * u if pname == "fp16x" else 40 * u)


def _lossy_problem(name, freqs, window):
    import phantoms as ph

    st, c_true = case(name)
    N = st.ring.n
    ab = lossy.Absorption(absorption_case(name, Y), Y)
    om = [2 * math.pi * f for f in freqs]
    dom = [om[0]] if len(om) == 1 else [om[1] - om[0]] * len(om)
    noise = ph.complex_noise((len(om), N, N), 2)
    data = ostep.synthesize(c_true, st, om, noise, "smooth", window, absorption=ab,
                            workers=WORKERS)
    return st, c_true, ab, om, dom, data


@pytest.mark.parametrize("name,window,mode", [("small", 1, 0), ("ring64", 1, 0),
                                              ("ragged", 5, 0), ("ragged", 5, 1)])
def test_frequency_step_lossy(ctx, name, window, mode):
    import torch

    freqs = [250e3] if name != "ragged" else [200e3, 260e3]
    st, c_true, ab, om, dom, data = _lossy_problem(name, freqs, window)
    c0 = np.full_like(c_true, C0)
    c_ref, parts = ostep.frequency_step(c0, st, om, dom, data, 0.12, window=window,
                                        mode="ray_born" if mode == 0 else "ray_only",
                                        return_parts=True, absorption=ab, workers=WORKERS)
    grid, ring, tp = abi_structs(st)
    _say(f"frequency_step_lossy {name} w={window} mode={mode}")
    c_g = _dev(c0.copy())
    rn = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ctx.frequency_step_lossy(grid, ring, tp, c_g, _dev(ab.alpha0), Y, window, om, dom,
                             _dev(data.astype(np.complex64)), 0.12, mode=mode, residual_norm=rn)
    c_new = to_np(c_g)
    q = st.grid.mask_index()
    err = rel_l2((c_new - c0).ravel()[q], (c_ref - c0).ravel()[q])
    _say(f"  rel L2 of the update {err:.2e}")
    assert err <= 1e-4
    outside = np.setdiff1d(np.arange(c0.size), q)
    assert np.all(c_new.ravel()[outside] == C0)
    rn_ref = sum(float(np.sum(np.abs(p["R"]) ** 2)) for p in parts["freqs"])
    assert abs(float(to_np(rn)[0]) - rn_ref) <= 1e-4 * rn_ref


@pytest.mark.parametrize("pname", ["bf16", "fp16", "fp16x"])
def test_frequency_step_lossy_lowp_image(ctx, pname):
    prec, u = LOWP[pname]
    name = "ring64"
    st, c_true, ab, om, dom, data = _lossy_problem(name, [250e3, 330e3], 1)
    c0 = np.full_like(c_true, C0)
    c_ref = ostep.frequency_step(c0, st, om, dom, data, 0.12, absorption=ab, workers=WORKERS)
    grid, ring, tp = abi_structs(st)
    _say(f"frequency_step_lossy {pname} {name}")
    c_g = _dev(c0.copy())
    ctx.frequency_step_lossy(grid, ring, tp, c_g, _dev(ab.alpha0), Y, 1, om, dom,
                             _dev(data.astype(np.complex64)), 0.12, prec=prec)
    q = st.grid.mask_index()
    c_new = to_np(c_g).ravel()[q]
    re = float(np.linalg.norm(c_new - c_ref.ravel()[q]) /
               np.linalg.norm((c_ref - c0).ravel()[q]))
    _say(f"  image RE {re:.2e}")
    assert re <= (IMAGE_GATE if pname == "fp16x" else 40 * u)


def test_alpha0_zero_gives_the_lossless_step(ctx):
    import phantoms as ph

    name = "ring64"
    st, c_true = case(name)
    N = st.ring.n
    om = [2 * math.pi * 250e3, 2 * math.pi * 330e3]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((2, N, N), 2), background="water",
                            workers=WORKERS)
    grid, ring, tp = abi_structs(st)
    c0 = np.full_like(c_true, C0)
    for prec in (1, 4):
        a = _dev(c0.copy())
        b = _dev(c0.copy())
        _say(f"lossless vs alpha0 = 0, prec {prec}")
        ctx.frequency_step(grid, ring, tp, a, 1, om, om, _dev(data.astype(np.complex64)), 0.12,
                           prec=prec)
        ctx.frequency_step_lossy(grid, ring, tp, b, _dev(np.zeros_like(c0)), Y, 1, om, om,
                                 _dev(data.astype(np.complex64)), 0.12, prec=prec)
        q = st.grid.mask_index()
        err = rel_l2((to_np(b) - c0).ravel()[q], (to_np(a) - c0).ravel()[q])
        _say(f"  rel L2 {err:.2e}")
        assert err <= 1e-6


def test_lossy_step_report_and_arguments(ctx):
    import torch
    from paper_2211_00316_amd import _lib

    name = "small"
    st, c_true, ab, om, dom, data = _lossy_problem(name, [250e3], 1)
    grid, ring, tp = abi_structs(st)
    c0 = np.full_like(c_true, C0)
    d = _dev(data.astype(np.complex64))
    for bad_y in (1.0, 0.0, 2.5, float("nan")):
        c_g = _dev(c0.copy())
        with pytest.raises(_lib.RayBornError) as e:
            ctx.frequency_step_lossy(grid, ring, tp, c_g, _dev(ab.alpha0), bad_y, 1, om, dom, d,
                                     0.12)
        assert e.value.status == _lib.RB_EINVAL
        assert np.array_equal(to_np(c_g), c0)
    # asynchronous form: the status goes to the device report
    rep = torch.zeros(_lib.REPORT_BYTES, dtype=torch.uint8, device="cuda:0")
    a = _dev(c0.copy())
    b = _dev(c0.copy())
    ctx.frequency_step_lossy(grid, ring, tp, a, _dev(ab.alpha0), Y, 1, om, dom, d, 0.12,
                             report=rep)
    ctx.frequency_step_lossy(grid, ring, tp, b, _dev(ab.alpha0), Y, 1, om, dom, d, 0.12)
    torch.cuda.synchronize()
    r = _lib.decode_report(rep)
    assert r.status == 0 and r.flags == 0 and r.ray_samples > 0
    assert torch.equal(a, b)
