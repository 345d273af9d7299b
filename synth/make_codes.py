"""Writes codes.json: the generator polynomial of each BCH code used by the
workloads, taken from the oracle's code construction (run from the repository
root: python -m synth.make_codes)."""
import json
import os

import oracle
from synth import CODES

out = {"source": "oracle BCH construction (narrow-sense primitive, zeros alpha^1..alpha^2t)",
       "codes": {}}
for name, (m, prim, t) in CODES.items():
    c = oracle.Code(m, prim, t)
    out["codes"][name] = {"m": m, "prim": prim, "t": t, "N": c.N, "K": c.K,
                          "g": [int(x) for x in c.g]}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "codes.json"), "w") as fh:
    json.dump(out, fh, indent=1)
print("wrote", list(out["codes"]))
