"""Write the stored oracle result of one shot of the gradient workload.

Calls only the FP64 oracle (``oracle/``) and the input generators
(``seisgen/``); nothing here touches the GPU library.  Run from the
repository root:

    python tests/golden/make_c4_golden.py            # about 2.3 h on one core
    python tests/golden/make_c4_golden.py fast       # the same with a 3 % faster true model

The workload is c4: a 200 x 200 x 160 model (h = 10 m) with a 20-cell sponge
(240 x 240 x 200 padded), 1200 steps, 2500 receivers, constant density.  The
stored shot is shot 1 at node (75, 67, 4).  Observed data are the oracle's
traces on the true model (background plus six +/-10 % blobs); the misfit and
gradient are taken at the starting model (the background).  That is the body
of Alg. 3 for one shot, evaluated end to end: J(v_start; d_obs = F(v_true)).

With the workload's own true model the residual is only 0.36 % of the data
and, at the receivers, zero until the reflections arrive (the direct wave
dominates both data sets): an FP32 propagator's rounding noise in the direct
wave, different in the observed and the synthetic run, then shows in the
shallow gradient at a few 1e-3.  The second file ("fast": the true model
scaled by 1.03, which moves every arrival) has a residual of the data's size
and tests the whole gradient at the 1e-3 level.

Stored (``c4_shot1.npz``):
  misfit              J (FP64)
  grad_norm           ||dJ/dv||_2 over the whole model
  grad_sketch[i]      <dJ/dv, r_i> for SKETCH seeded standard-normal volumes
                      r_i (numpy default_rng(SKETCH_SEED + i), float32 draws)
  grad_z60            dJ/dv on model plane z = 60 (every x-tile seam crosses it)
  grad_y100           dJ/dv on model plane y = 100 (x-z section)
  illum_norm          ||I||_2 of the source illumination sum_n (w^n)^2
  illum_z60           the illumination on plane z = 60
  trace_ids           receivers whose traces are stored
  seis, dobs          their synthetic (start model) and observed traces
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import seisgen  # noqa: E402

SHOT = 1
SKETCH = 32
SKETCH_SEED = 20250217
TRACE_IDS = np.arange(0, 2500, 157)  # 16 receivers spread over the surface grid
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "c4_shot1.npz")
# true-model scale -> stored file
CASES = {"": (1.0, OUT), "fast": (1.03, os.path.join(HERE, "c4_shot1_fast.npz"))}


def sketch_vector(i, shape):
    return np.random.default_rng(SKETCH_SEED + i).standard_normal(shape, dtype=np.float32)


def main(case=""):
    scale, out = CASES[case]
    start = seisgen.workload("c4_start")
    true = start.extra["v_true"] * scale
    g = oracle.Grid(**start.grid_kwargs())
    src = start.sources[SHOT]
    t0 = time.time()
    print(f"observed data on the true model: {g.padded_shape}, {g.nt} steps", flush=True)
    dobs = oracle.forward(g, true, None, start.wavelet, src, start.receivers).seis
    dobs = dobs.astype(np.float32)
    print(f"  {time.time() - t0:.0f} s; gradient at the start model", flush=True)
    ref = oracle.gradient(g, start.vel, None, start.wavelet, src, start.receivers, dobs,
                          illumination=True)
    print(f"  {time.time() - t0:.0f} s; J = {ref.misfit:.6e}", flush=True)
    grad = ref.grad
    sk = np.array([float(np.sum(grad * sketch_vector(i, grad.shape).astype(np.float64)))
                   for i in range(SKETCH)])
    np.savez_compressed(
        out,
        misfit=np.float64(ref.misfit),
        grad_norm=np.float64(np.linalg.norm(grad)),
        grad_sketch=sk,
        grad_z60=grad[60].astype(np.float32),
        grad_y100=grad[:, 100, :].astype(np.float32),
        illum_norm=np.float64(np.linalg.norm(ref.illum)),
        illum_z60=ref.illum[60].astype(np.float32),
        trace_ids=TRACE_IDS.astype(np.int32),
        seis=ref.seis[TRACE_IDS].astype(np.float32),
        dobs=dobs[TRACE_IDS],
        shot=np.int32(SHOT),
        true_scale=np.float64(scale),
    )
    print(f"wrote {out} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "")
