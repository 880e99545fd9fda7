"""Writes rising_bubble_2d_fd.json: central finite differences of the oracle
for the differentiation workload (D2Q9 rising bubble 256x512, radius 24 at
y = 64, density ratio 100, viscosity ratio 10, g 1e-5, sigma 5e-3; loss L =
gas centroid height with the smoothed Heaviside), with every decision of the
perturbed runs replayed from the unperturbed one (the frozen-decision
program that the reverse mode differentiates).

Calls only the oracle.  Steps: sigma (1 +- h) (h relative: an absolute
1e-4 is 2% of sigma) and phi0 +- h v, v standard normal on the band
(numpy default_rng(12345)), zero elsewhere.  h = 1e-4 after 500 steps;
after 2000 steps the largest h whose replayed runs stay in the linear range
is 1e-6 (with h = 1e-5 the replayed sigma (1 - h) run leaves it: L moves by
0.8), checked by repeating the differences at h / 10.

Run: python tests/golden/make_rising_bubble_fd.py  (about 5 minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2601_05936_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rising_bubble_2d_fd.json")


def band_direction(phi0, band, seed=12345):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(phi0.shape)
    v[np.abs(phi0) >= band] = 0.0
    return v


def main():
    w = W.rising_bubble_2d(storage=W.F64)
    p = w["params"]
    phi0 = w["phi0"]
    v = band_direction(phi0, p["band"])
    sig = p["sigma"]
    res = {"_cite": "finite differences of the oracle with replayed decisions; see the generator's docstring",
           "workload": w["name"], "axis": 1, "cases": []}
    for steps, h in ((500, 1e-4), (2000, 1e-6)):
        base = O.Oracle(p, phi0, record=True)
        base.step(steps)
        L0 = float(base.integrals()["centroid"][1])

        def run(q, ph):
            o = O.Oracle(q, ph, replay=base)
            o.step(steps)
            assert not o.replay_failed()
            return float(o.integrals()["centroid"][1])

        fd = {}
        for hh in (h, h / 10):
            Ls = [run(dict(p, sigma=sig * (1 + s * hh)), phi0) for s in (1, -1)]
            Lv = [run(p, phi0 + s * hh * v) for s in (1, -1)]
            fd[hh] = ((Ls[0] - Ls[1]) / (2 * hh * sig), (Lv[0] - Lv[1]) / (2 * hh))
            print(steps, hh, fd[hh], flush=True)
        (ds, dv), (ds10, dv10) = fd[h], fd[h / 10]
        # in the linear range to within the gate of the checks (1e-4)
        assert abs(ds - ds10) < 1e-4 * abs(ds10) and abs(dv - dv10) < 1e-4 * abs(dv10), fd
        res["cases"].append({"steps": steps, "h": h, "L": L0, "dL_dsigma": ds, "dL_dphi0_dot_v": dv,
                             "h_over_10": {"dL_dsigma": ds10, "dL_dphi0_dot_v": dv10},
                             "v": "default_rng(12345).standard_normal on |phi0| < band"})
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
