"""Write horn_4m_counts.json: eigenvalue counts N(omega) = #{omega_j < omega}
of the 752,845-DOF horn pencil (synth.horn.horn_pencil(16, 2604), seed 2) by
the oracle's inertia count (Sylvester's law, oracle/inertia.py).  Run from the
repository root: python tests/golden/make_horn_counts.py  (about 2 minutes)."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import inertia  # noqa: E402
from synth.horn import horn_pencil  # noqa: E402

OMEGAS = [200.0, 205.0, 210.0, 215.0, 220.0, 230.0, 240.0, 250.0, 300.0, 400.0, 600.0]


def main():
    S, m = horn_pencil(16, 2604)
    counts = {}
    for om in OMEGAS:
        counts[repr(om)] = inertia.count_below(S, m, om * om)
        print(om, counts[repr(om)], flush=True)
    out = {
        "what": "number of eigenvalues omega^2 < omega_key^2 of the horn_4m pencil (16 x 16 cross-section, 2604 "
                "layers, 5% jitter, seed 2), Neumann, lumped P1",
        "source": "oracle.inertia.count_below (banded LDL^T, Sylvester's law of inertia)",
        "n": int(S.shape[0]),
        "nnz": int(S.nnz),
        "counts": counts,
    }
    with open(os.path.join(ROOT, "tests", "golden", "horn_4m_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
