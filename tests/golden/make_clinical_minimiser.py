"""Writes clinical_minimiser.json: the FP64 oracle's minimiser of the
clinical workload (256x256x128 at 1.5 x 1.5 x 2.5 mm, K = 3, 512x384 at
0.8 mm, step 0.75 mm, 1% noise, the seeded phantom of synth.clinical, every
input rounded to float32 as the GPU receives it), with and without the
intensity fit (Eq. A.1), and the tumour position there.

Calls only the oracle and the seeded input generators; takes a few minutes
on a CPU.  Run from the repository root:

    python tests/golden/make_clinical_minimiser.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1102_1712_amd import synth  # noqa: E402


def main():
    c = synth.clinical()
    # the measured image as the FP32 solve receives it (f0, mean and U are
    # already rounded to the case's type)
    y = O.measured_projection(c.vol, c.proj, c.f0, c.mean, c.U, c.w_star, c.xi, c.noise_level)
    y = y.astype(np.float32).astype(np.float64)
    out = {"_source": "FP64 oracle (oracle.minimise: plain CG, then Newton's method on the "
                      "gradient to ||g|| <= 1e-10 ||g0||) on synth.clinical(); "
                      "written by tests/golden/make_clinical_minimiser.py",
           "workload": c.name, "angle": c.proj.angle, "w_star": list(map(float, c.w_star))}
    for fit in (True, False):
        prob = O.Problem(c.vol, c.proj, c.f0, c.mean, c.U, y, fit_intensity=fit)
        w, info = O.minimise(prob, np.zeros(c.K))
        loc, it = O.locate(c.vol, c.mean, c.U, w, c.tumour_c0)
        out["fit" if fit else "nofit"] = {
            "w": list(map(float, w)), "J": info["J"], "a": info["a"], "b": info["b"],
            "cg_iters": info["cg"].iters, "newton_steps": info["newton_steps"],
            "gnorm_rel": info["gnorm"] / info["gnorm0"],
            "hessian_eigs": list(map(float, info["hessian_eigs"])),
            "tumour_mm": list(map(float, loc))}
        print(fit, out["fit" if fit else "nofit"], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "clinical_minimiser.json"),
              "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
