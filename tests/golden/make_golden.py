"""Writes the stored expected values under tests/golden/.

Every value here comes from the CPU oracle (``oracle/``) on seeded inputs from
``gen/``; nothing is taken from the GPU library.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from gen import blocks_to_dense, config_matrix  # noqa: E402
from oracle.refinement import coefficients, irsi, lif, true_residual  # noqa: E402


def main():
    S, cfg = config_matrix(0)
    D = blocks_to_dense(S)
    lam = np.linalg.eigvalsh(D)
    Z, info, c = irsi(D, S.b, 0.0, m=4, start="inv_sqrt_lmax", start_value=float(lam[-1]))
    Zl, plan = lif(D, S.b, 0.0, m=4, base_rows=128)
    out = {
        "source": "oracle/ on gen.config_matrix(0): water, 100 molecules, n=700, b=32, tau=0",
        "coefficients_m4": coefficients(4),
        "lambda_min": float(lam[0]),
        "lambda_max": float(lam[-1]),
        "irsi_inv_sqrt_lmax": {"c": c, "iterations": info.iterations, "norms": info.norms,
                               "true_residual": true_residual(D, Z)},
        "lif_base128": {"top_iterations": plan.info.iterations, "top_norms": plan.info.norms,
                        "true_residual": true_residual(D, Zl)},
    }
    with open(os.path.join(HERE, "water100_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
