"""Writes ``psi_scale.json``: the deformation-potential amplitude of the
moving-mesh workload for each grid size.

The unit-variance potential ``psi`` (seed 1, ``P ~ k^-4 exp(-(k/(16*2pi))^2)``)
is multiplied by the largest ``s`` for which every cell of
``J = I + Hess(s psi)`` has ``0.3 <= det J <= 3`` and positive eigenvalues
(admissibility, Sec. 4.2; bisection as in App. C, eq. bisection), computed by
the CPU oracle only.  Run from the repository root:
``python tests/golden/make_psi_scale.py``.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mg_oracle as O  # noqa: E402
from workloads import psi_unit     # noqa: E402


def main(sizes=(8, 16, 32, 64, 128, 256)):
    out = {}
    for n in sizes:
        s = O.admissible_scale(psi_unit(n), 1.0 / n)
        out[str(n)] = s
        print(n, s, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "psi_scale.json")
    with open(path, "w") as f:
        json.dump({"det_range": [0.3, 3.0], "seed": 1, "h": "1/n", "scale": out}, f, indent=1)


if __name__ == "__main__":
    main()
