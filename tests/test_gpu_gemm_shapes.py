"""Parity of the 16-bit contractions at intermediate, ragged shapes: several row slabs of
256 transducers (an odd count, a last slab of a single K step of 32, rows past the padded
row length inside a slab), node counts that are not multiples of the 128-node tile. The
whole output is compared with the FP64 oracle.

Operands are seeded 16-bit values (random sign, magnitude in [0.5, 1)), exact in BF16 and
FP16, so both sides take identical inputs and only the FP32 accumulation of the GPU
differs; the residual is complex symmetric with BF16-exact entries, so the
back-projection's symmetrised, power-of-two scaled operand is exact too."""
import math
import sys

import numpy as np
import pytest

from oracle import born
from tests.gpu_cases import rel_l2, to_np

pytestmark = pytest.mark.gpu

# (transducers, mask nodes): slabs of 256 rows of R' and K steps of 32 transducers
SHAPES = [
    (280, 1000),   # two slabs, the second one K step long
    (600, 777),    # three slabs (a middle one), padded rows 608.. past the last slab's data
    (513, 300),    # three slabs, one row in the last
]
PRECS = ["bf16", "fp16"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_00316_amd import _lib

    return _lib.Context("cuda:0")


def _values(shape, seed, positive=False):
    """Seeded BF16 tensor (host): random sign (or +), magnitude in [0.5, 1)."""
    import torch

    n = int(np.prod(shape))
    g = torch.Generator().manual_seed(seed)
    words = torch.randint(-2 ** 63, 2 ** 63 - 1, ((n + 3) // 4,), dtype=torch.int64, generator=g)
    bits = (words.view(torch.int16)[:n] & (0x007F if positive else -0x7F81)) | 0x3F00
    return bits.view(torch.bfloat16).reshape(shape)


def _prec(pname):
    import torch
    from paper_2211_00316_amd import _lib

    return {"bf16": (_lib.RB_BF16, torch.bfloat16), "fp16": (_lib.RB_F16, torch.float16)}[pname]


@pytest.mark.parametrize("pname", PRECS)
@pytest.mark.parametrize("N,Pm", SHAPES)
def test_born_forward_shapes(ctx, N, Pm, pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec, dt = _prec(pname)
    _say(f"born_forward {pname} N={N} n_mask={Pm}")
    gr = _lib.Green.empty(N, Pm, "cuda:0", prec)
    gr.G.zero_()
    re = _values((N, Pm), 51, positive=True)
    im = _values((N, Pm), 52)
    gr.G[0, :, :Pm].copy_(re.to(dt))
    gr.G[1, :, :Pm].copy_(im.to(dt))
    d = to_np(ctx.born_forward(gr, None, None))
    assert np.array_equal(d, d.T)
    G = re.double().numpy() + 1j * im.double().numpy()
    ref = born.forward(G, np.ones(Pm), np.ones(Pm))
    err = rel_l2(d, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("pname", PRECS)
@pytest.mark.parametrize("N,Pm", SHAPES)
def test_backproject_shapes(ctx, N, Pm, pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec, dt = _prec(pname)
    _say(f"backproject {pname} N={N} n_mask={Pm}")
    gr = _lib.Green.empty(N, Pm, "cuda:0", prec)
    gr.G.zero_()
    gr.H.zero_()
    host = [_values((Pm, N), 61 + k) for k in range(6)]  # (component, part) planes
    for k in range(6):
        gr.H[k // 2, k % 2, :, :N].copy_(host[k].to(dt))
    a = _values((N, N), 71).float().numpy() + 1j * _values((N, N), 72).float().numpy()
    R = np.triu(a) + np.triu(a, 1).T  # complex symmetric
    rng = np.random.default_rng(73)
    cq = 1450.0 + 100.0 * rng.random(Pm)
    om = 2 * math.pi * 300e3
    dm = to_np(ctx.backproject(gr, torch.as_tensor(R.astype(np.complex64), device="cuda:0"),
                               torch.as_tensor(cq, device="cuda:0"), om, 0.5 * om))
    Hs = [(host[2 * k].double().numpy() + 1j * host[2 * k + 1].double().numpy()).T
          for k in range(3)]
    S = born.backproject_weight(om, 0.5 * om, cq)
    ref = born.backproject(R.astype(np.complex128), Hs[0], Hs[1], Hs[2], S)
    err = rel_l2(dm, ref)
    _say(f"  rel L2 {err:.2e}")
    assert err <= 1e-5
