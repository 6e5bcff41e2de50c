"""rb_backproject_noalloc, the allocation-free form of rb_backproject (its scratch in the
library's fixed device array): the same result as rb_backproject through the C ABI, on two
calls in a row with the second on a smaller problem, and a size beyond the array rejected
before any launch."""
import ctypes
import math
import sys

import numpy as np
import pytest

from tests.gpu_cases import C0, case, oracle_tables, rel_l2, tables_to_gpu, to_np

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(ctx, name, prec, seed):
    import torch

    st, c = case(name)
    om = 2 * math.pi * 350e3
    tb_o, _ = oracle_tables(name)
    gr = ctx.build_green(tables_to_gpu(tb_o), om, C0, prec=prec)
    N = st.ring.n
    rng = np.random.default_rng(seed)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    cq = c.ravel()[st.grid.mask_index()]
    return (gr, torch.as_tensor(R, device="cuda:0"), torch.as_tensor(cq, device="cuda:0"), om)


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16"])
def test_noalloc_backprojection_matches_backproject(pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"f32": _lib.RB_F32, "bf16": _lib.RB_BF16, "fp16": _lib.RB_F16}[pname]
    ctx = _lib.Context("cuda:0")
    # the larger problem first, then a smaller one: the second call reuses the scratch that
    # the first left behind
    for name, seed in (("ring64", 9), ("small", 10)):
        gr, R, cq, om = _problem(ctx, name, prec, seed)
        _say(f"noalloc back-projection {pname} {name} n={gr.n} n_mask={gr.n_mask}")
        ref = to_np(ctx.backproject(gr, R, cq, om, 0.5 * om))
        out = torch.full((gr.n_mask,), float("nan"), dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        ctx.backproject_noalloc(gr, R, cq, om, 0.5 * om, out)
        got = to_np(out)
        assert np.all(np.isfinite(got))
        assert rel_l2(got, ref) <= 1e-6
        assert np.array_equal(got, ref)   # the same kernels on the same values
        # accumulate form: adds to what the caller passes
        ctx.backproject_noalloc(gr, R, cq, om, 0.5 * om, out, accumulate=True)
        assert rel_l2(to_np(out), 2 * ref) <= 1e-6
    ctx.close()


def test_noalloc_backprojection_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_2211_00316_amd import _lib

    ctx = _lib.Context("cuda:0")
    lib = _lib.load()
    tiny = torch.zeros(16, dtype=torch.float32, device="cuda:0")
    # n = 4096 transducers over 10^6 nodes: about 140 MB of scratch; rejected by the size check
    # before anything reads the (deliberately tiny) operands
    g = _lib._Green(4096, 1_000_000, _lib.RB_BF16, tiny.data_ptr(), tiny.data_ptr(),
                    tiny.data_ptr())
    st = lib.rb_backproject_noalloc(ctx._h, ctypes.byref(g), ctypes.c_void_p(tiny.data_ptr()),
                                    ctypes.c_void_p(tiny.data_ptr()), 1e6, 1e5,
                                    ctypes.c_void_p(tiny.data_ptr()), 0)
    assert st == _lib.RB_EINVAL
    assert b"scratch" in lib.rb_last_error(ctx._h)
    torch.cuda.synchronize()
    assert torch.count_nonzero(tiny).item() == 0
    ctx.close()
