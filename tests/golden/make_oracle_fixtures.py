"""Write the stored oracle results that the GPU parity tests compare against.

    python tests/golden/make_oracle_fixtures.py [--threads N]

Every value written here comes from the CPU oracle (oracle/) on the seeded
synthetic 30-atom, 270-function molecule (molgen workload "w30"; the gradient
workload uses the same geometry and density):
  * w30_jk_tol1e-10.npz  -- J and K (upper triangles, row-major) at Schwarz
                            tolerance 1e-10, and the number of kept quartets;
  * w30_grad_atoms.npz   -- rows of dE/dR at tolerance 1e-10 for a heavy atom and
                            a hydrogen (exact rows: the oracle differentiates the
                            selected atoms over every quartet that touches them).
Run times on 8 host threads: about 5 and 10 minutes.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_11185_amd import molgen  # noqa: E402

GRAD_ATOMS = [3, 20]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", choices=["jk", "grad"], default=None)
    a = ap.parse_args()
    mol = molgen.workload("w30")
    iu = np.triu_indices(mol.n_bf)
    if a.only in (None, "jk"):
        t = time.time()
        J, K, kept = oracle.jk(mol, 1e-10, nthreads=a.threads)
        np.savez_compressed(os.path.join(HERE, "w30_jk_tol1e-10.npz"), J_upper=J[0][iu],
                            K_upper=K[0][iu], n_bf=mol.n_bf, tol=1e-10, kept=kept)
        print(f"w30 J/K: {kept} quartets, {time.time() - t:.0f} s", flush=True)
    if a.only in (None, "grad"):
        t = time.time()
        G = oracle.grad(mol, 1e-10, nthreads=a.threads, atoms=GRAD_ATOMS)
        np.savez_compressed(os.path.join(HERE, "w30_grad_atoms.npz"), atoms=np.array(GRAD_ATOMS),
                            G=G[:, GRAD_ATOMS, :], tol=1e-10)
        print(f"w30 gradient rows {GRAD_ATOMS}: {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
