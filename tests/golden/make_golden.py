"""Writes c1_oracle.json: oracle outputs for the 2D n=32 single-bump workload.

Calls only the oracle and the seeded input generators."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.solve import OracleProblem  # noqa: E402

w = synth.workload("c1")
prob = OracleProblem(w["n"], w["d"], w["omega"], w["m"], b=2)
res = prob.solve(w["uI"][0])
out = {
    "workload": "2D n=32 omega=8pi single Gaussian bump, b=2, tol 1e-8, restart 30",
    "iters": res.iters,
    "relres": res.relres,
    "sigma_min": [st.sigma_min for st in prob.stencils],
    "k0": [prob.ktab[0, 0].real, prob.ktab[0, 0].imag],
    "u_norm": float(abs(res.x @ res.x.conj()) ** 0.5),
}
json.dump(out, open(os.path.join(os.path.dirname(__file__), "c1_oracle.json"), "w"), indent=1)
print(out)
