"""How far rounding alone moves a long oracle run: the FP64 oracle with the
Tucker operators applied in the order mu = 1..d against the same run with the
order reversed (d..1).  Both orders give the same operator (mode products along
different directions commute, Sec. 2 eq. (5)), so their distance measures the
sensitivity of the scheme's trajectory to rounding, the floor under any
GPU-vs-oracle comparison of the same run.

    python tests/mode_order_drift.py fhn3d 200 50      # 128^3, 200 steps, every 50
    python tests/mode_order_drift.py brusselator3d 100 20

Prints, at each checkpoint, the relative infinity-norm distance per component.
Only calls the oracle and the input generator.
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth as S  # noqa: E402

BUILDERS = {"fhn3d": S.fhn_3d, "brusselator3d": S.brusselator_3d,
            "schnakenberg2d": S.schnakenberg_2d}


def main():
    name, steps, every = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    n = int(sys.argv[4]) if len(sys.argv) > 4 else None
    w = BUILDERS[name]() if n is None else BUILDERS[name](n)
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    rev = tuple(reversed(range(w.d)))
    a = (U0, V0)
    b = (U0, V0)
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        a = O.solve(*a, p, k, mats=mats)
        b = O.solve(*b, p, k, mats=mats, order=rev)
        done += k
        eu = O.rel_inf_error(b[0], a[0])
        ev = O.rel_inf_error(b[1], a[1])
        print(f"{w.name} {'x'.join(map(str, w.n))} step {done}: reversed-order drift "
              f"u={eu:.3e} v={ev:.3e} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
