"""Write tests/golden/exact_ising.json: exact (e, C_V) for the lattices the
statistical tests and the benchmark use.  Calls only oracle.exact_ising."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact_ising as ex  # noqa: E402

CASES = [(L, b) for L in (16, 32, 64) for b in (0.4, ex.BETA_C)] + [(1024, 0.4), (4096, 0.4), (4096, ex.BETA_C)]


def main():
    values = []
    for L, b in CASES:
        e, c = ex.exact(L, b)
        values.append({"L": L, "beta": b, "e": e, "C_V": c})
        print(L, b, e, c, flush=True)
    out = {"source": "oracle/exact_ising.py (Kaufman / Ferdinand-Fisher torus partition function)",
           "values": values}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_ising.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
