"""Writes tests/golden/ring256_grid512_steps.npz: the FP64 oracle's first frequency steps of
the 256-transducer workload (ring of 110 mm, 512^2 grid at 0.45 mm, breast-like phantom with
3 lesions, frequencies 100-800 kHz low to high, 720 rays per transducer), for the GPU parity
tests of that workload. Calls only oracle/ (and the seeded input generators of phantoms/).

Steps follow the frequency continuation of Section 6.3.2: step k uses the k-th frequency
alone (Delta omega = the list's spacing), the smoothing window of its quartile, tau = 0.12,
and starts from the model the previous step produced (water for the first). The measured
data are the oracle's ray-Born prediction of the phantom about its smoothed map (same
window) plus 1 % complex Gaussian noise. The steps trace the smoothed map rounded to FP32,
the representation the GPU path receives it in (rounding the map alone moves the direction
of the second step by 1.05e-4 and its predicted data by 1.6e-5, relative). Stored (float32 /
complex64, the GPU's own types):
  data[k]   measured data of frequency k, complex64 [N][N];
  pred[k]   predicted data of step k's start model at frequency k on the valid pairs with
            e != r (zero elsewhere), complex64 [N][N];
  dc[k]     c - c0 on the mask nodes after step k, float32 [P_m];
  dm[k]     the step's direction delta m on the mask nodes, float32 [P_m];
  grad[k]   the Q = 1 gradient Re J^H g_res of the step's residual (Eq. functional-gradient,
            w = omega^2 h^2), float32 [P_m];
  rn[k]     sum |g_res|^2 of the step, float64;
  windows, freqs_hz, tau.
Usage: python tests/golden/make_ring256_grid512.py [--steps 3] [--workers 8]
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import phantoms as ph  # noqa: E402
from oracle import born, step as ostep  # noqa: E402
from oracle.medium import Grid, Ring  # noqa: E402

OUT = os.path.join(HERE, "ring256_grid512_steps.npz")


def setup():
    w = ph.MEDIUM
    grid = Grid(w.nx, w.ny, w.dx, w.x0, w.y0, w.mask_radius)
    st = ostep.StepSetup(grid, Ring(w.n_trans, w.radius, w.psi0), w.n_rays, w.ds, w.max_steps())
    return w, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    w, st = setup()
    K = args.steps
    N = w.n_trans
    q = st.grid.mask_index()
    c_true = ph.phantom_for(w)
    oms = [2 * math.pi * f for f in w.freqs[:K]]
    dom = 2 * math.pi * (w.freqs[1] - w.freqs[0])
    wins = [w.smooth_window(k) for k in range(K)]
    noise = ph.complex_noise((K, N, N), w.noise_seed)
    t0 = time.time()
    data = np.zeros((K, N, N), dtype=np.complex128)
    for win in sorted(set(wins)):
        ks = [k for k in range(K) if wins[k] == win]
        data[ks] = ostep.synthesize(c_true, st, [oms[k] for k in ks], noise[ks],
                                    background="smooth", window=win, workers=args.workers)
    print(f"data of {K} frequencies: {time.time() - t0:.0f} s", flush=True)
    c = np.full_like(c_true, ph.C_WATER)
    out = dict(data=data.astype(np.complex64), pred=[], dc=[], dm=[], grad=[], rn=[],
               windows=np.array(wins), freqs_hz=np.array(w.freqs[:K]), tau=np.array(w.tau))
    for k in range(K):
        t0 = time.time()
        c_new, parts = ostep.frequency_step(c, st, [oms[k]], [dom], data[k:k + 1], w.tau,
                                            window=wins[k], return_parts=True,
                                            workers=args.workers, map32=True)
        f = parts["freqs"][0]
        keep = parts["tables"].rx_valid & ~np.eye(N, dtype=bool)
        out["pred"].append(np.where(keep, f["g"], 0).astype(np.complex64))
        out["dc"].append((c_new.ravel()[q] - ph.C_WATER).astype(np.float32))
        out["dm"].append(parts["dm"].astype(np.float32))
        wq = np.full(q.size, oms[k] ** 2 * w.dx ** 2)
        out["grad"].append(born.adjoint(f["G"], wq, f["R"]).astype(np.float32))
        out["rn"].append(float(np.sum(np.abs(f["R"]) ** 2)))
        c = c_new
        print(f"step {k}: {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, **{k: np.asarray(v) for k, v in out.items()})
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
