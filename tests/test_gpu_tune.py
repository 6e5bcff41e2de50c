"""Autotuned forward launches (rb_autotune, rb_set_tuning): the tuner times every candidate
tile and K split and keeps the fastest; every configuration it may choose gives the Born
forward term of the FP64 oracle on the same operands (only the order of the FP32 partial
sums changes); a tuned frequency step still matches the oracle; invalid tunings are refused
before anything runs."""
import math
import sys

import numpy as np
import pytest

from oracle import born
from tests.gpu_cases import C0, abi_structs, case, rel_l2, to_np

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _operand(n, n_mask, pname, seed):
    """Seeded G rounded to the operand type on the host, as GPU green record and as the
    complex values the oracle takes."""
    import torch
    from paper_2211_00316_amd import _lib

    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n_mask)) + 1j * rng.standard_normal((n, n_mask))
    if pname == "f32":
        Gq = G.astype(np.complex64)
        gr = _lib.Green.empty(n, n_mask, "cuda:0", _lib.RB_F32)
        gr.G.copy_(torch.as_tensor(Gq))
        return gr, Gq.astype(np.complex128)
    prec = {"bf16": _lib.RB_BF16, "f16": _lib.RB_F16}[pname]
    dt = torch.bfloat16 if pname == "bf16" else torch.float16
    re = torch.as_tensor(G.real).to(dt)
    im = torch.as_tensor(G.imag).to(dt)
    gr = _lib.Green.empty(n, n_mask, "cuda:0", prec)
    gr.G.zero_()
    gr.G[0, :, :n_mask].copy_(re)
    gr.G[1, :, :n_mask].copy_(im)
    return gr, re.double().numpy() + 1j * im.double().numpy()


@pytest.mark.parametrize("pname", ["bf16", "f32"])
def test_every_tuned_configuration_matches_the_oracle(ctx, pname):
    # 300 transducers (a ragged last tile row) over 5000 nodes (ragged K): both tiles of the
    # 16-bit forward and K splits 1 .. 64 (more chunks than K steps is clamped).
    from paper_2211_00316_amd import _lib

    n, n_mask = 300, 5000
    gr, Gq = _operand(n, n_mask, pname, 11)
    prec = gr.prec
    ref = born.forward(Gq, np.ones(n_mask), np.ones(n_mask))
    tiles = [_lib.RB_TILE_128x128] if pname == "f32" else [_lib.RB_TILE_256x128,
                                                           _lib.RB_TILE_128x128]
    for tile in tiles:
        for spk in (1, 3, 8, 24, 64, 1024):
            ctx.set_tuning({"n": n, "n_mask": n_mask, "prec": prec, "fwd_tile": tile,
                            "fwd_splitk": spk})
            d = to_np(ctx.born_forward(gr, None, None))
            err = rel_l2(d, ref)
            _say(f"{pname} tile {tile} splitk {spk}: rel L2 {err:.2e}")
            assert err <= 1e-5 and np.array_equal(d, d.T)
    ctx.set_tuning(None)
    assert ctx.get_tuning(n, n_mask, prec) is None


@pytest.mark.parametrize("pname", ["bf16", "f32"])
def test_autotune_keeps_the_fastest_and_the_step_still_matches(ctx, pname):
    import torch
    import phantoms as ph
    from oracle import step as ostep
    from paper_2211_00316_amd import _lib

    prec = {"bf16": _lib.RB_BF16, "f32": _lib.RB_F32}[pname]
    st, c_true = case("ring64")
    grid, ring, tp = abi_structs(st)
    t = ctx.autotune(grid, ring, prec)
    _say(f"autotune {pname} ring64: {t.as_dict()}")
    assert t.n == st.ring.n and t.n_mask == st.grid.mask_index().size and t.prec == prec
    # K splits 8 .. 64 or the built-in one (which may be larger for small n)
    assert t.fwd_ms > 0 and 1 <= t.fwd_splitk <= 1024
    assert ctx.get_tuning(t.n, t.n_mask, prec).as_dict() == t.as_dict()
    N = st.ring.n
    om = [2 * math.pi * 250e3]
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((1, N, N), 2), background="water")
    c0 = np.full_like(c_true, C0)
    c_ref = ostep.frequency_step(c0, st, om, om, data, 0.12)
    c_g = torch.as_tensor(c0.copy(), device="cuda:0")
    ctx.frequency_step(grid, ring, tp, c_g, 1, om, om,
                       torch.as_tensor(data.astype(np.complex64), device="cuda:0"), 0.12,
                       prec=prec)
    q = st.grid.mask_index()
    c_new = to_np(c_g).ravel()[q]
    if pname == "f32":
        err = rel_l2(c_new - C0, (c_ref - c0).ravel()[q])
        _say(f"  tuned step: update rel L2 {err:.2e}")
        assert err <= 1e-4
    else:
        # image error relative to the step's change: 40 units of BF16 rounding
        err = rel_l2(c_new - C0, (c_ref - c0).ravel()[q])
        _say(f"  tuned step: image RE {err:.2e} "
             f"(||c||-normalised {rel_l2(c_new, c_ref.ravel()[q]):.2e})")
        assert err <= 40 * 2.0 ** -9
    ctx.set_tuning(None)


def test_invalid_tunings_are_refused(ctx):
    from paper_2211_00316_amd import _lib

    good = {"n": 64, "n_mask": 1000, "prec": _lib.RB_BF16, "fwd_tile": _lib.RB_TILE_256x128,
            "fwd_splitk": 8}
    for bad in ({"fwd_splitk": 0}, {"fwd_splitk": 2000}, {"fwd_tile": 7}, {"n": 0},
                {"prec": _lib.RB_F32}, {"prec": 9}):
        with pytest.raises(_lib.RayBornError) as e:
            ctx.set_tuning({**good, **bad})
        assert e.value.status == _lib.RB_EINVAL
    assert ctx.get_tuning(64, 1000, _lib.RB_BF16) is None
    ctx.set_tuning(good)
    ctx.set_tuning({**good, "prec": _lib.RB_F16, "fwd_splitk": 16})
    assert ctx.get_tuning(64, 1000, _lib.RB_BF16).fwd_splitk == 8
    assert ctx.get_tuning(64, 1000, _lib.RB_F16).fwd_splitk == 16
    ctx.set_tuning(None)
    assert ctx.get_tuning(64, 1000, _lib.RB_F16) is None
