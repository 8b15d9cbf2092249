"""The host symmetric eigensolver of the Davidson driver (csrc/symeig.h:
Householder tridiagonalisation + implicit QL), built with g++ and checked
against LAPACK (numpy.linalg.eigh) and the defining identities A V = V diag(w),
V^T V = I, on random, degenerate, diagonal, zero and tridiagonal matrices."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_04346_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("symeig") / "symeig_driver")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", exe,
                           os.path.join(ROOT, "tests", "symeig_driver.cpp")])
    return exe


def solve(exe, A):
    n = A.shape[0]
    inp = f"{n}\n" + "\n".join(f"{x:.17g}" for x in A.ravel()) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    assert out[0] == "1"
    w = np.array(out[1:1 + n], float)
    V = np.array(out[1 + n:], float).reshape(n, n)
    return w, V


def cases():
    rng = np.random.default_rng(0)
    out = []
    for n in (1, 2, 3, 7, 40, 200):
        M = rng.standard_normal((n, n))
        out.append((f"random{n}", M + M.T))
    Q, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    out.append(("degenerate", Q @ np.diag([1.0] * 12 + [-2.0] * 8 + [5.0] * 4) @ Q.T))
    out.append(("diagonal", np.diag([3.0, 1.0, 2.0, 1.0, 3.0, 0.0])))
    out.append(("zero", np.zeros((5, 5))))
    out.append(("tridiagonal", 2 * np.eye(30) - np.eye(30, k=1) - np.eye(30, k=-1)))
    # a Davidson-like projected matrix: a few well-separated low values above a dense cluster
    G = np.diag(np.concatenate([[-93.5, -91.0, -90.8], -80 + rng.standard_normal(29)]))
    X = 1e-3 * rng.standard_normal((29, 3))
    G[3:, :3] = X
    G[:3, 3:] = X.T
    out.append(("davidson-like", G))
    return out


@pytest.mark.parametrize("name,A", cases(), ids=[c[0] for c in cases()])
def test_sym_eig(driver, name, A):
    w, V = solve(driver, A)
    n = A.shape[0]
    scale = max(1.0, np.abs(A).max())
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() <= 1e-12 * scale * max(n, 1)
    assert np.abs(A @ V - V * w).max() <= 1e-12 * scale * max(n, 1)
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12 * max(n, 1)
