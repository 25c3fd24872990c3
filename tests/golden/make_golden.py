"""Writes exact_iterates.json: IBMI iterates in exact rational arithmetic (eq. (IBMI),
Algorithm 1, identity initial guess) for three tiny matrices.  Calls only the oracle."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

CASES = [
    {"name": "p2_two_singletons", "A": [[2, 1], [1, 2]], "sets": [[0], [1]], "sweeps": 3},
    {"name": "p3_overlapping_pairs", "A": [[4, 1, 1], [1, 3, 1], [1, 1, 2]],
     "sets": [[0, 1], [1, 2]], "sweeps": 2},
    {"name": "p4_two_pairs", "A": [[4, 1, 0, 1], [1, 4, 1, 0], [0, 1, 4, 1], [1, 0, 1, 4]],
     "sets": [[0, 1], [2, 3]], "sweeps": 2},
    {"name": "p5_three_overlapping", "A": [[5, 1, 0, 1, 0], [1, 4, 1, 0, 1], [0, 1, 6, 2, 0],
                                            [1, 0, 2, 5, 1], [0, 1, 0, 1, 3]],
     "sets": [[0, 1, 2], [2, 3], [3, 4]], "sweeps": 2},
]

out = {"source": "eq. (IBMI) and Algorithm 1 applied in exact rational arithmetic "
                 "by oracle.exact_ibmi; identity initial guess", "cases": []}
for c in CASES:
    its = oracle.exact_ibmi(c["A"], c["sets"], c["sweeps"])
    out["cases"].append({"name": c["name"], "A": c["A"], "sets": c["sets"],
                         "iterates": [[[str(x) for x in row] for row in h] for h in its]})
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_iterates.json"), "w") as f:
    json.dump(out, f, indent=1)
