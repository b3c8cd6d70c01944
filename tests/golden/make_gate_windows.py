"""Writes ``and_gate_window.txt``: the range of passive-gap excitability for
which the generated coincidence-detector AND gate (Sec. 4.1) fires on input 11
but not on 10 or 01, found by scanning the FP64 oracle.  Calls only the
oracle and the input generators.

    python tests/golden/make_gate_windows.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1901_06535_amd import inputs  # noqa: E402


def fires(wl):
    r = oracle.run_workload(wl, track_arrival=True)
    x0, x1, y0, y1 = wl.extra["probe"]
    return bool((r.arrival[y0:y1, x0:x1] < oracle.NEVER).any())


def main():
    ok = []
    for pg in np.round(np.arange(0.1150, 0.1351, 0.0005), 4):
        res = [fires(inputs.and_case(i, phi_gap=float(pg))) for i in ((1, 0), (0, 1), (1, 1))]
        if res == [False, False, True]:
            ok.append(float(pg))
    lo, hi = min(ok), max(ok)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "and_gate_window.txt")
    with open(out, "w") as fh:
        fh.write("# AND gate (Sec. 4.1), generated geometry of inputs.and_case, workload\n"
                 "# parameters (eps=0.022, D_u=1.0, rest of Table 1), background 0.2.\n"
                 "# Passive-gap phi range (scan step 0.0005) where 10 -> 0, 01 -> 0, 11 -> 1\n"
                 "# on the FP64 oracle.  Written by make_gate_windows.py.\n")
        fh.write("lo %.4f\nhi %.4f\n" % (lo, hi))
    print(lo, hi)


if __name__ == "__main__":
    main()
