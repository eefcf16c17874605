"""Write oracle-only sampled elements of sigma = A X at full size (calls synth and oracle only).

usage: python tests/golden/make_sigma_rows_golden.py chainring1000 [workers]
Writes tests/golden/<name>_sigma_rows.json: sigma_m,ia for a seeded block of 30 trial vectors
(synth.random_trial_vectors(30, nocc, nvir, seed)) at a fixed sample of rows (i, a), computed by
oracle.risp.sigma_rows in FP64 straight from the integrals (no factor is stored, so the 1000-atom
case fits in host memory). The chunks of auxiliary shells run in a pool of worker processes; the AO
transition densities sit in a memory-mapped temporary file that the workers share.
"""
import json
import multiprocessing as mp
import os
import shutil
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import risp as R  # noqa: E402

M_VECTORS = 30

_W = {}


def sample_rows(nocc, nvir, nvir_k, seed, n_random=56):
    """Row sample: seeded random (i, a) plus the corners and both sides of the window edge."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    edge = [(0, 0), (0, nvir_k - 1), (0, nvir_k), (nocc - 1, 0), (nocc - 1, nvir - 1), (nocc // 2, nvir_k - 1),
            (nocc // 2, nvir_k), (nocc - 1, nvir_k - 1)]
    rnd = [(int(i), int(a)) for i, a in zip(rng.integers(0, nocc, n_random), rng.integers(0, nvir, n_random))]
    rows = sorted({i * nvir + a for i, a in edge + rnd})
    return np.array(rows, dtype=np.int64)


def _init(mol, prm, mask, dpath, dshape):
    _W.update(mol=mol, prm=prm, mask=mask, D=np.memmap(dpath, dtype=np.float64, mode="r", shape=dshape))


def _run(args):
    k, (kind, idx, ri, ra) = args
    out = R.sigma_rows_chunk(_W["mol"], _W["prm"], _W["mask"], kind, idx, _W["D"], ri, ra)
    return k, out


def main(name, workers=4):
    t0 = time.time()
    mol = synth.config_system(name)
    prm = R.Params()
    auxJ, _ = R.select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    pairs, mask, _ = R.schwarz_pairs(mol.coords, mol.shells, auxJ, prm.schwarz_tau)
    occK, virK = R.window_sets(mol.mo_energy, mol.nocc, prm.window_ev, prm.window_mode)
    nocc, nvir = mol.nocc, mol.nvir
    X = synth.random_trial_vectors(M_VECTORS, nocc, nvir, mol.seed)
    rows = sample_rows(nocc, nvir, len(virK), mol.seed)
    print(f"{name}: nao={mol.nao} nocc={nocc} nvir={nvir} pairs={len(pairs)} nvK={len(virK)} rows={len(rows)} "
          f"({time.time() - t0:.0f}s)", flush=True)
    tmp = tempfile.mkdtemp(prefix="risp_golden_")
    try:
        dpath = os.path.join(tmp, "D.f64")
        nao = mol.nao
        D = np.memmap(dpath, dtype=np.float64, mode="w+", shape=(M_VECTORS, nao, nao))
        Co, Cv = mol.mo_coeff[:, :nocc], mol.mo_coeff[:, nocc:]
        for k in range(M_VECTORS):  # D_k = C_occ X_k C_vir^T
            D[k] = (Co @ X[k]) @ Cv.T
        D.flush()
        del D
        print(f"densities written ({time.time() - t0:.0f}s)", flush=True)
        ctx = mp.get_context("spawn")
        os.environ["OPENBLAS_NUM_THREADS"] = "2"  # read by the workers' BLAS at start-up
        with ctx.Pool(workers, initializer=_init,
                      initargs=(mol, prm, mask, dpath, (M_VECTORS, nao, nao))) as pool:
            def run_chunks(tasks, _D, ri, ra):
                res = [None] * len(tasks)
                jobs = [(k, (kind, idx, ri, ra)) for k, (kind, idx) in enumerate(tasks)]
                for done, (k, out) in enumerate(pool.imap_unordered(_run, jobs)):
                    res[k] = out
                    if done % 25 == 24 or done == len(tasks) - 1:
                        print(f"chunks {done + 1}/{len(tasks)} ({time.time() - t0:.0f}s)", flush=True)
                return res

            S = R.sigma_rows(mol, X, rows, prm, pair_mask=mask, run_chunks=run_chunks)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    out = {
        "workload": name, "seed": mol.seed, "nao": mol.nao, "nocc": nocc, "nvir": nvir, "params": prm.__dict__,
        "npair": int(len(pairs)), "nocc_k": int(len(occK)), "nvir_k": int(len(virK)),
        "x": f"synth.random_trial_vectors({M_VECTORS}, nocc, nvir, {mol.seed})",
        "rows": [int(r) for r in rows], "sigma": [[float(v) for v in S[m]] for m in range(M_VECTORS)],
        "seconds": time.time() - t0, "workers": workers,
        "source": "oracle/risp.py sigma_rows (FP64) on the synth generator; no GPU value enters this file",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_sigma_rows.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 4)
