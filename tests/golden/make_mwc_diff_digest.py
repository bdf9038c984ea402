"""Writes mwc_diff_multipliers.json: SHA-256 digests of the oracle's first
2^20 and 2^21 MWC_DIFF multipliers (little-endian uint32, decreasing), with
the last multiplier of each prefix.  Calls only the oracle (its threaded
enumeration of the downward search)."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    a = oracle.mwc_multipliers(1 << 21, threads=os.cpu_count() or 1)
    rec = {}
    for n in (1 << 20, 1 << 21):
        rec[str(n)] = {"sha256": hashlib.sha256(a[:n].astype("<u4").tobytes()).hexdigest(), "last": int(a[n - 1])}
    with open(os.path.join(HERE, "mwc_diff_multipliers.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(rec)


if __name__ == "__main__":
    main()
