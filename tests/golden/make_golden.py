"""Writes the oracle-derived golden files of this directory.

Calls only the CPU oracle (oracle/) on the seeded generators (gen/); nothing
here touches the GPU library.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402


def uniform1000():
    p = gen.make_uniform(n=1000, nev=100, nex=40)
    ev, v, r, st = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    return {
        "source": "oracle.solve on gen.make_uniform(n=1000, nev=100, nex=40, deg=20, tol=1e-10)",
        "iterations": st.iterations, "matvecs": st.matvecs, "locked": st.locked,
        "b_sup": st.b_sup, "evals": [float(x) for x in ev],
        "max_resid": float(r.max()),
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_uniform1000.json")
    with open(out, "w") as f:
        json.dump(uniform1000(), f, indent=1)
    print("wrote", out)
