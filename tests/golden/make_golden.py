"""Write oracle-only reference values for the larger parity cases (calls synth and oracle only).

usage: python tests/golden/make_golden.py chainring300
Writes tests/golden/<name>_oracle.json with the lowest excitation energies of the FP64 oracle
(block Davidson, residual tolerance 1e-7) for the default method parameters.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import risp as R  # noqa: E402


def main(name, nstates=15, tol=1e-7):
    t0 = time.time()
    mol = synth.config_system(name)
    prm = R.Params()
    F = R.build_factors(mol, prm)
    t1 = time.time()
    print(f"factors {t1 - t0:.1f}s naux_j={F.B_ia.shape[0]} naux_k={F.Bx_ij.shape[0]} "
          f"noK={len(F.occK)} nvK={len(F.virK)} pairs={len(F.pairs)}", flush=True)
    # the diagonal of A as guess and preconditioner: same eigenpairs, far fewer iterations
    r = R.davidson(F, nstates, tol=tol, block=min(2 * nstates, 30), diag=R.diag_A(F), verbose=True)
    t2 = time.time()
    print(f"davidson {t2 - t1:.1f}s iters={r.iters} converged={r.converged}", flush=True)
    out = {
        "workload": name, "seed": mol.seed, "nao": mol.nao, "nocc": mol.nocc, "nvir": mol.nvir,
        "params": prm.__dict__, "nstates": nstates, "tol": tol, "converged": bool(r.converged),
        "energies_ha": [float(x) for x in r.energies],
        "residuals": [float(x) for x in r.resid[-1]],
        "npair": int(len(F.pairs)), "nocc_k": int(len(F.occK)), "nvir_k": int(len(F.virK)),
        "cond_S": float(mol.cond_S), "seconds": {"factors": t1 - t0, "davidson": t2 - t1},
        "source": "oracle/risp.py (FP64) on the synth generator; no GPU value enters this file",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, np.array(out["energies_ha"]))


if __name__ == "__main__":
    main(sys.argv[1])
