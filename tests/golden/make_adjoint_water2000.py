"""Writes tests/golden/adjoint_water2000.json: sampled entries of the exact-limit
derivatives at the differentiation workload's full size (water-2000, n = 14000,
b = 64, tau = 0, S dense), for L = tr(G^T Z) with G = N(0, 1) on Z's block
pattern (seed 1003):

* IRSI: sym(dL/dS) of Z = S^{-1/2} (oracle.adjoint.inv_sqrt_grad, one dense
  eigendecomposition);
* LIF (4096-row leaves): sym(dL/dS) of the recursive limit
  Z = Z_0 (Z_0^T S Z_0)^{-1/2} with inverse Cholesky leaves
  (oracle.adjoint.lif_limit_grad).

Stored: 2000 entries (i, j) drawn with seed 77, the Frobenius norm and the
largest magnitude of each derivative, and <dS, E_k> for the three symmetric
unit directions E_k on S's pattern (seeds 2030, 2031, 2032) -- the
directional derivatives a finite-difference check takes.  Every value comes
from oracle/ on inputs from gen/; nothing from the GPU library.  Takes several
minutes of dense eigendecompositions.  Run from the repository root:
    python tests/golden/make_adjoint_water2000.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from gen import blocks_to_dense, config_matrix, random_on_pattern, random_symmetric_on_pattern  # noqa: E402
from oracle.adjoint import inv_sqrt_grad, lif_limit_grad  # noqa: E402


def main():
    S, cfg = config_matrix(3)
    D = blocks_to_dense(S)
    G = blocks_to_dense(random_on_pattern(S, 1003))
    E = [blocks_to_dense(random_symmetric_on_pattern(S, 2030 + k)) for k in range(3)]
    rng = np.random.default_rng(77)
    ii = rng.integers(0, S.n, 2000)
    jj = rng.integers(0, S.n, 2000)
    out = {"source": "oracle.adjoint on gen.config_matrix(3): water, 2000 molecules, n=14000, b=64, tau=0; "
                     "G = gen.random_on_pattern(S, 1003); E_k = gen.random_symmetric_on_pattern(S, 2030 + k)",
           "n": int(S.n), "i": ii.tolist(), "j": jj.tolist()}
    for name, fn in (("irsi", lambda: inv_sqrt_grad(D, G)), ("lif", lambda: lif_limit_grad(D, G, 64, 4096))):
        t0 = time.time()
        dS = fn()
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
        out[name] = {"values": dS[ii, jj].tolist(), "fro": float(np.linalg.norm(dS)),
                     "max_abs": float(np.max(np.abs(dS))),
                     "directional": [float(np.sum(dS * e)) for e in E]}
        del dS
    with open(os.path.join(HERE, "adjoint_water2000.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
