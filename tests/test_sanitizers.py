"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU: the oracle (oracle/oracle.c: sigma, diagonal, density matrices,
matrix elements), the library's host Slater-Condon rules (csrc/hmat.hip, the
P-space and cisigma_hmat_block) and the host eigensolver (csrc/symeig.h).  Each
sanitized build must run clean (any report aborts it) and agree with the
ordinary build (the oracle library, and the oracle for the host rules)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_04346_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

SPACES = [(6, 3, 3, None), (7, 2, 4, None), (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])), (5, 0, 2, None)]


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    ora = str(d / "oracle_san")
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-std=c99", "-o", ora,
                           os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"), "-lm"])
    hm = str(d / "hmat_san")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I", CSRC, "-o", hm,
                           os.path.join(ROOT, "tests", "sanitize_hmat_driver.cpp"),
                           os.path.join(CSRC, "hmat.hip")])
    se = str(d / "symeig_san")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-I", CSRC, "-o", se,
                           os.path.join(ROOT, "tests", "symeig_driver.cpp")])
    return ora, hm, se


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    return np.array(r.stdout.split(), dtype=float)


def _fmt(a):
    return "\n".join(f"{x:.17g}" for x in np.ravel(a))


@pytest.mark.parametrize("case", SPACES, ids=lambda c: f"n{c[0]}a{c[1]}b{c[2]}" + ("gas" if c[3] else ""))
def test_oracle_sanitized(builds, case):
    norb, na, nb, gas = case
    h, g = si.integrals(norb, 2 * norb, 2)
    sp = oracle.Space(norb, na, nb, h, g, gas=gas)
    c = si.ci_vector(sp.ndet, 3)
    gn, mn, mx = gas if gas else ([norb], [na + nb], [na + nb])
    text = f"{norb} {na} {nb} {len(gn)}\n{' '.join(map(str, gn))}\n{' '.join(map(str, mn))}\n" \
           f"{' '.join(map(str, mx))}\n{_fmt(h)}\n{_fmt(g)}\n{_fmt(c)}\n"
    out = _run(builds[0], text)
    nd = int(out[0])
    assert nd == sp.ndet
    o = 1
    sig, hd = out[o:o + nd], out[o + nd:o + 2 * nd]
    o += 2 * nd
    n2 = norb * norb
    r1, r2 = out[o:o + n2], out[o + n2:o + n2 + n2 * n2]
    o += n2 + n2 * n2
    assert np.allclose(sig, sp.sigma(c), rtol=0, atol=1e-12)
    assert np.allclose(hd, sp.hdiag(), rtol=0, atol=1e-12)
    w1, w2 = sp.rdm(c)
    assert np.allclose(r1, np.ravel(w1), atol=1e-12) and np.allclose(r2, np.ravel(w2), atol=1e-12)
    idx = np.arange(0, nd, 7)
    want = [sp.h_elem(i, (i * 13 + 5) % nd) for i in idx]
    assert np.allclose(out[o:], want, rtol=0, atol=1e-12)


def test_host_rules_sanitized(builds):
    """The library's host Slater-Condon rules under the sanitizers, against the
    oracle's matrix elements on every pair of a small space with n_a != n_b."""
    norb, na, nb = 7, 3, 2
    h, g = si.integrals(norb, 14, 4)
    sp = oracle.Space(norb, na, nb, h, g)
    dets = sp.dets()
    rng = np.random.default_rng(5)
    pairs = [(i, j) for i in range(sp.ndet) for j in range(sp.ndet) if rng.random() < 0.05 or abs(i - j) < 3]
    lines = "\n".join(f"{dets[i][0]} {dets[i][1]} {dets[j][0]} {dets[j][1]}" for i, j in pairs)
    out = _run(builds[1], f"{norb}\n{_fmt(h)}\n{_fmt(g)}\n{len(pairs)}\n{lines}\n")
    want = np.array([sp.h_elem(i, j) for i, j in pairs])
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_symeig_sanitized(builds):
    rng = np.random.default_rng(6)
    for n in (1, 5, 33):
        M = rng.standard_normal((n, n))
        A = M + M.T
        out = _run(builds[2], f"{n}\n{_fmt(A)}\n")
        assert out[0] == 1
        w = out[1:1 + n]
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-10)
