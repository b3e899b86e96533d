"""Write tests/golden/oracle_unet_samples.json: the FP64 U-Net reference
(oracle/unet.py) at the production gather's shape, for the GPU forward's
full-size parity test.

Network: P = 32 model panels, base 16 (1,225,345 parameters), He-normal
weights plus N(0, 0.02^2) on every parameter (nonzero biases), rounded to FP32,
drawn from numpy's default_rng(seed).  Input: the blended gather of the
1024-sample x 256-trace workload (``synth.workload("crg-1024x256-nv32")``),
traces as rows (H = 256, W = 1024), divided by its RMS and rounded to FP32,
which is how the warm start feeds the network.

Stored: the output norms and values at seeded sample positions, once for the
exact network and once under the oracle's BF16 operand precision model; the
relative L2 distance between the two whole outputs (what BF16 operands alone
cost at this shape), and between the BF16-operand network summed in FP64 and
in FP32 (the floor of an FP32-accumulating BF16 implementation).

Calls only ``oracle`` and ``synth``.  Usage:
    python tests/golden/make_unet_values.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import unet as U  # noqa: E402
from synth import make_gather, workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_unet_samples.json")
N_SAMPLES = 2048
WORKLOAD = "crg-1024x256-nv32"
P, BASE, SEED = 32, 16, 21


def inputs():
    """(spec, theta, x) of the stored case; the GPU test rebuilds them with
    this same function."""
    spec = U.UNetSpec(cin=1, pout=P, base=BASE)
    rng = np.random.default_rng(SEED)
    theta = U.init_params(spec, rng) + 0.02 * rng.standard_normal(spec.n_params())
    theta = theta.astype(np.float32).astype(np.float64)
    d = make_gather(workload(WORKLOAD)).d_blend
    x = (d / np.sqrt(np.mean(d * d))).astype(np.float32).astype(np.float64)
    return spec, theta, x[None, None]


def main():
    spec, theta, x = inputs()
    out = {"workload": WORKLOAD, "pout": P, "base": BASE, "seed": SEED, "H": x.shape[2], "W": x.shape[3],
           "n_params": spec.n_params()}
    srng = np.random.default_rng(SEED + 1)
    mi = srng.integers(0, P * x.shape[2] * x.shape[3], N_SAMPLES)
    wi = srng.integers(0, x.shape[2] * x.shape[3], N_SAMPLES)
    out["y_m_index"], out["y_w_index"] = mi.tolist(), wi.tolist()
    res = {}
    for tag, bf in (("exact", False), ("bf16", True)):
        t0 = time.time()
        y_m, y_w, _ = U.forward(spec, theta, x, bf16=bf)
        print(f"{tag}: {time.time() - t0:.0f} s", flush=True)
        res[tag] = (y_m, y_w)
        out[f"{tag}_y_m_norm"] = float(np.linalg.norm(y_m))
        out[f"{tag}_y_w_norm"] = float(np.linalg.norm(y_w))
        out[f"{tag}_y_m_value"] = y_m.ravel()[mi].tolist()
        out[f"{tag}_y_w_value"] = y_w.ravel()[wi].tolist()
    (em, ew), (bm, bw) = res["exact"], res["bf16"]
    out["bf16_cost_y_m"] = float(np.linalg.norm(bm - em) / np.linalg.norm(em))
    out["bf16_cost_y_w"] = float(np.linalg.norm(bw - ew) / np.linalg.norm(ew))
    print(f"BF16 operand cost: y_m {out['bf16_cost_y_m']:.2e}  y_w {out['bf16_cost_y_w']:.2e}", flush=True)
    fm, fw, _ = U.forward(spec, theta, x, bf16=True, acc32=True)
    out["acc32_floor_y_m"] = float(np.linalg.norm(fm - bm) / np.linalg.norm(bm))
    out["acc32_floor_y_w"] = float(np.linalg.norm(fw - bw) / np.linalg.norm(bw))
    print(f"FP32-accumulation floor: y_m {out['acc32_floor_y_m']:.2e}  y_w {out['acc32_floor_y_w']:.2e}",
          flush=True)
    tmp = OUT + ".tmp"
    json.dump(out, open(tmp, "w"))
    os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
