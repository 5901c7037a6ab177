"""Write the oracle's singular values for the full-size configurations.

Calls only the FP64 CPU oracle (oracle/) on the seeded matrices of testmats
and stores, per configuration, sigma (17 significant digits), the column-
scaled condition number kappa_s used by the e_sigma gate, the sweep count
and the sha256 of A's column-major bytes (so a reader can confirm the input
was regenerated bit for bit).  Usage:
    python tests/golden/make_oracle_sigma.py [C2 C3a C3b]
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import testmats  # noqa: E402
from testmats import metrics  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
GEN = {"C2": testmats.config_c2, "C3a": testmats.config_c3a, "C3b": testmats.config_c3b}


def sha_of(A: np.ndarray) -> str:
    return hashlib.sha256(np.asfortranarray(A).tobytes(order="F")).hexdigest()


def fingerprint(A: np.ndarray) -> list:
    """Frobenius norm and eight fixed entries of A: the seeded input is
    regenerated with LAPACK/BLAS calls whose last bits depend on the host CPU,
    so a regenerated A is compared to these with a relative tolerance (the
    sigma gate absorbs perturbations of that size)."""
    m, n = A.shape
    idx = [(0, 0), (m - 1, n - 1), (m // 2, n // 3), (m // 3, n // 2), (1, n - 2), (m - 2, 1),
           (m // 5, 4 * n // 5), (4 * m // 5, n // 5)]
    return [float(np.linalg.norm(A))] + [float(A[i, j]) for i, j in idx]


def main(names):
    oracle.set_threads(os.cpu_count() or 1)
    for name in names:
        t0 = time.time()
        A, _ = GEN[name]()
        U, S, V, info = oracle.svd(A, order="rr")
        ks = metrics.kappa_s(A)
        dt = time.time() - t0
        path = os.path.join(HERE, f"oracle_sigma_{name}.txt")
        with open(path, "w") as f:
            f.write(f"# oracle sigma for {name}: {A.shape[0]} x {A.shape[1]}\n")
            f.write(f"# sha256(A column-major) {sha_of(A)}\n")
            f.write("# fingerprint " + " ".join(f"{x:.17g}" for x in fingerprint(A)) + "\n")
            f.write(f"# kappa_s {ks:.17g}\n")
            f.write(f"# oracle status {info['status']} sweeps {info['sweeps']} order rr\n")
            f.write("# written by tests/golden/make_oracle_sigma.py (calls only oracle/)\n")
            for s in S:
                f.write(f"{s:.17g}\n")
        print(f"{name}: {dt:.0f}s sweeps={info['sweeps']} kappa_s={ks:.3e}", flush=True)


def load(name):
    """(sigma, kappa_s, fingerprint, sweeps) from a stored file."""
    path = os.path.join(HERE, f"oracle_sigma_{name}.txt")
    fp = ks = None
    sweeps = None
    vals = []
    with open(path) as f:
        for line in f:
            if line.startswith("# fingerprint"):
                fp = [float(x) for x in line.split()[2:]]
            elif line.startswith("# kappa_s"):
                ks = float(line.split()[-1])
            elif line.startswith("# oracle status"):
                sweeps = int(line.split()[5])
            elif not line.startswith("#"):
                vals.append(float(line))
    return np.array(vals), ks, fp, sweeps


if __name__ == "__main__":
    main(sys.argv[1:] or ["C2", "C3a", "C3b"])
