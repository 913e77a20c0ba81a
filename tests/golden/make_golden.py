"""Write the stored exact references under tests/golden/ (calls only oracle/).

exact_lngE.json: ln g(E) of the periodic L x L Ising model (J = 1) for
L in {4, 6, 8, 12, 16, 24, 32}, indexed by e = (E + 2N)/4, null where g(E) = 0,
from Kaufman's closed form (oracle/exact.py; the exact reference of Sec. 3,
Fig. 5 of the paper, after Beale).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def main(sizes=(4, 6, 8, 12, 16, 24, 32)):
    out = {"what": "ln g(E) of the periodic LxL Ising model, e = (E+2N)/4",
           "source": "oracle/exact.py (Kaufman closed form, integer coefficients)",
           "lattices": {}}
    for L in sizes:
        g = exact.exact_gE(L)
        out["lattices"][str(L)] = {
            "N": L * L,
            "lnge": [None if v == 0 else math.log(v) for v in g],
        }
        print("L =", L, "done", flush=True)
    with open(os.path.join(HERE, "exact_lngE.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
