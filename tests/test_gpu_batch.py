"""Frequency steps of several scans in one call (rb_frequency_step_batch) and the serving loop
on top of it: each scan's result against the FP64 oracle step, identical to the same scan
stepped alone (the grouped launches compute per problem what a single launch computes), a
failing scan isolated from the others (conditions forced from the host), and the
continuous-batching server: each request's model the same alone and in the mix."""
import functools
import math
import sys

import numpy as np
import pytest

from oracle import step as ostep
from tests.gpu_cases import C0, abi_structs, case, rel_l2, to_np

pytestmark = pytest.mark.gpu

# (parity case, frequencies of the step, smoothing window): scans of different N and grids
SCANS = {"small": ([250e3], 1), "ragged": ([200e3, 260e3], 5), "folded": ([250e3], 3),
         "ring64": ([300e3], 1)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def _scan(name):
    """(setup, omegas, spacings, window, data, oracle step from water) of a scan."""
    import phantoms as ph

    st, c_true = case(name)
    freqs, window = SCANS[name]
    om = [2 * math.pi * f for f in freqs]
    dom = [om[0]] if len(om) == 1 else [om[1] - om[0]] * len(om)
    data = ostep.synthesize(c_true, st, om, ph.complex_noise((len(om), st.ring.n, st.ring.n), 2),
                            background="water")
    c0 = np.full_like(c_true, C0)
    c_ref = ostep.frequency_step(c0, st, om, dom, data, 0.12, window=window)
    return st, om, dom, window, data, c_ref


def _contexts(n):
    import torch
    from paper_2211_00316_amd import _lib

    return [_lib.Context("cuda:0", stream=torch.cuda.Stream()) for _ in range(n)]


def _step_args(ctx, name, tp=None):
    import torch
    from paper_2211_00316_amd import _lib

    st, om, dom, window, data, _ = _scan(name)
    grid, ring, tp0 = abi_structs(st)
    c = torch.full((st.grid.ny, st.grid.nx), C0, dtype=torch.float64, device="cuda:0")
    d = torch.as_tensor(data.astype(np.complex64), device="cuda:0")
    return _lib.ScanStep(ctx, grid, ring, tp or tp0, c, window, om, dom, d, 0.12)


def _alone(name, prec):
    import torch

    ctx = _contexts(1)[0]
    s = _step_args(ctx, name)
    torch.cuda.synchronize()
    ctx.frequency_step(s.grid, s.ring, s.tp, s.c, s.smooth_w, s.omegas, s.d_omegas, s.data,
                       s.tau, prec=prec)
    torch.cuda.synchronize()
    ctx.close()
    return s.c


@pytest.mark.parametrize("pname", ["f32", "bf16", "fp16x"])
def test_batch_matches_oracle_and_single_steps(pname):
    import torch
    from paper_2211_00316_amd import _lib

    prec = {"f32": _lib.RB_F32, "bf16": _lib.RB_BF16, "fp16x": _lib.RB_F16X}[pname]
    names = ["small", "ragged", "folded", "ring64"]
    ctxs = _contexts(len(names))
    steps = [_step_args(cx, n) for cx, n in zip(ctxs, names)]
    torch.cuda.synchronize()
    _say(f"batch {pname} of {names}")
    status = _lib.frequency_step_batch(steps, prec)
    assert status == [_lib.RB_OK] * len(names)
    for name, s in zip(names, steps):
        alone = _alone(name, prec)
        _say(f"  {name}: batch == alone {torch.equal(s.c, alone)}")
        assert torch.equal(s.c, alone), name
        if name in ("small", "ragged"):
            st, *_, c_ref = _scan(name)
            q = st.grid.mask_index()
            c = to_np(s.c).ravel()[q]
            if pname == "f32":
                err = rel_l2(c - C0, (c_ref.ravel() - C0)[q])
                _say(f"  {name}: update rel L2 vs oracle {err:.2e}")
                assert err <= 1e-4
            else:
                # image error relative to the step's change (split form: the 2e-3 tolerance
                # of the reduced-precision form; BF16: 40 units of its rounding)
                err = rel_l2(c - C0, (c_ref.ravel() - C0)[q])
                _say(f"  {name}: image RE vs oracle {err:.2e} "
                     f"(||c||-normalised {rel_l2(c, c_ref.ravel()[q]):.2e})")
                assert err <= (2e-3 if pname == "fp16x" else 40 * 2.0 ** -9)
    for cx in ctxs:
        cx.close()


def test_batch_isolates_a_failing_scan():
    # One scan's max_steps is too small for its rays to reach the ring: that scan reports
    # RB_ENONFINITE and keeps its model; the others commit the same result as alone.
    import torch
    from paper_2211_00316_amd import _lib

    ctxs = _contexts(3)
    st, *_ = _scan("ragged")
    _, _, tp = abi_structs(st)
    short = _lib.TraceParams(tp.n_rays, 10, tp.ds, tp.c0)
    steps = [_step_args(ctxs[0], "small"), _step_args(ctxs[1], "ragged", tp=short),
             _step_args(ctxs[2], "ring64")]
    torch.cuda.synchronize()
    _say("batch with a failing scan")
    status = _lib.frequency_step_batch(steps, _lib.RB_BF16)
    assert status == [_lib.RB_OK, _lib.RB_ENONFINITE, _lib.RB_OK]
    assert torch.all(steps[1].c == C0)
    assert torch.equal(steps[0].c, _alone("small", _lib.RB_BF16))
    assert torch.equal(steps[2].c, _alone("ring64", _lib.RB_BF16))
    for cx in ctxs:
        cx.close()


def test_batch_rejects_invalid_arguments_before_launch():
    import torch
    from paper_2211_00316_amd import _lib

    ctx = _contexts(1)[0]
    a, b = _step_args(ctx, "small"), _step_args(ctx, "small")
    with pytest.raises(_lib.RayBornError) as e:
        _lib.frequency_step_batch([a, b], _lib.RB_BF16)     # one context twice
    assert e.value.status == _lib.RB_EINVAL
    with pytest.raises(ValueError):
        _lib.frequency_step_batch([], _lib.RB_BF16)
    assert torch.all(a.c == C0) and torch.all(b.c == C0)
    ctx.close()


def test_step_bytes_covers_what_a_context_allocates():
    # The admission estimate is an upper bound of the device memory a step takes.
    import torch
    from paper_2211_00316_amd import _lib

    st, *_ = _scan("ring64")
    grid, ring, tp = abi_structs(st)
    budget = 1 << 28
    est = _lib.step_bytes(grid, ring, tp, _lib.RB_BF16, budget)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = _contexts(1)[0]
    ctx.set_sample_budget(budget)
    s = _step_args(ctx, "ring64")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _lib.frequency_step_batch([s], _lib.RB_BF16)
    torch.cuda.synchronize()
    used = free1 - torch.cuda.mem_get_info()[0]
    _say(f"step_bytes {est}, context took {used} (free before the context {free0})")
    assert est > 0 and used <= est + (8 << 20)   # allocator granularity
    ctx.close()


def test_server_alone_equals_mix():
    # Four requests of different scans and step counts; three wait at time 0, the fourth
    # arrives during the first batch and joins at a step boundary. Every request's final
    # model must equal the one it reaches when served alone.
    import torch
    from paper_2211_00316_amd import _lib, serve

    def requests(arrivals):
        out = []
        for rid, (name, n_steps) in enumerate([("small", 3), ("ragged", 2), ("ring64", 2),
                                               ("folded", 3)]):
            st, om, dom, window, data, _ = _scan(name)
            grid, ring, tp = abi_structs(st)
            d = torch.as_tensor(data.astype(np.complex64), device="cuda:0")
            # one frequency per step: the scan's first frequency, repeated
            dd = d[:1].repeat(n_steps, 1, 1).contiguous()
            c0 = torch.full((st.grid.ny, st.grid.nx), C0, dtype=torch.float64, device="cuda:0")
            out.append(serve.Request(rid, arrivals[rid], grid, ring, tp, [om[0]] * n_steps,
                                     [dom[0]] * n_steps, [window] * n_steps, dd, c0, 0.12,
                                     tag=name))
        return out

    ex = serve.GpuExecutor(_lib.RB_BF16, sample_budget=1 << 28)
    budget = 8 << 30
    mix = serve.Server(ex, budget).run(requests([0.0, 0.0, 0.0, 1e-4]))
    _say(f"mix: {mix.summary()}")
    assert all(r.status == 0 and r.steps_done == r.n_steps for r in mix.requests)
    assert max(mix.batches) >= 3 and mix.requests[3].t_admit > 0
    assert mix.peak_bytes <= budget
    for r in mix.requests:
        alone = serve.Server(ex, budget).run([requests([0.0] * 4)[r.rid]]).requests[0]
        _say(f"  request {r.rid} ({r.tag}): alone == mix {torch.equal(alone.c, r.c)}")
        assert torch.equal(alone.c, r.c), r.tag
        assert torch.isfinite(r.c).all()
