"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test targets a different way the oracle could be wrong:
  * brute force: Eq. 6 built literally from second-quantised operators in the
    full Fock space (Jordan-Wigner signs), projected on the oracle's
    determinants -> catches any dropped term, wrong sign, wrong index or
    transposed integral in the Slater-Condon rules;
  * two-site Hubbard closed form; non-interacting closed form;
  * spin symmetry [H, S^2] = 0 and alpha<->beta transposition symmetry;
  * GAS: unrestricted GAS = CAS (Sec. 4: GAS partitioning without restrictions
    does not truncate the expansion) and restricted GAS = projected CAS;
  * determinant counts against numbers printed in the paper and an
    independent itertools enumeration of the ordering contract;
  * Davidson against dense eigh.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent brute force: Fock-space operators with Jordan-Wigner signs
# ---------------------------------------------------------------------------
def _fock_ops(nso):
    dim = 1 << nso
    cre = []
    for so in range(nso):
        rows, cols, vals = [], [], []
        for x in range(dim):
            if not (x >> so) & 1:
                sign = -1.0 if bin(x & ((1 << so) - 1)).count("1") % 2 else 1.0
                rows.append(x | (1 << so))
                cols.append(x)
                vals.append(sign)
        cre.append(sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim)))
    ann = [c.T.tocsr() for c in cre]
    return cre, ann


def _brute_h(norb, h, g):
    """Eq. 6 with E_kl of Eq. 7: sum h_kl E_kl + 1/2 sum (ij|kl)(E_ij E_kl - d_jk E_il).
    Spin orbital index: alpha p -> p, beta p -> norb + p."""
    cre, ann = _fock_ops(2 * norb)
    n = norb
    E = [[cre[k] @ ann[l] + cre[n + k] @ ann[n + l] for l in range(n)] for k in range(n)]
    H = sp.csr_matrix((1 << (2 * n), 1 << (2 * n)))
    for k in range(n):
        for l in range(n):
            if h[k, l] != 0:
                H = H + h[k, l] * E[k][l]
    for i in range(n):
        for j in range(n):
            EE = None
            for k in range(n):
                for l in range(n):
                    v = g[i, j, k, l]
                    if v == 0:
                        continue
                    term = E[i][j] @ E[k][l]
                    if j == k:
                        term = term - E[i][l]
                    EE = term * v if EE is None else EE + term * v
            if EE is not None:
                H = H + 0.5 * EE
    return H.tocsr(), cre


def _det_state(norb, abits, bbits, cre):
    """alpha-hat(I_a) beta-hat(I_b)|vac>: creation operators in ascending orbital
    order, alpha string to the left (Eq. 2)."""
    ops = [p for p in range(norb) if (abits >> p) & 1] + [norb + p for p in range(norb) if (bbits >> p) & 1]
    v = np.zeros(1 << (2 * norb))
    v[0] = 1.0
    for so in reversed(ops):
        v = cre[so] @ v
    return v


def _oracle_vs_brute(norb, na, nb, seed, gas=None):
    h, g = si.integrals(norb, 2 * norb, seed)
    S = oracle.Space(norb, na, nb, h, g, gas=gas)
    Hb, cre = _brute_h(norb, h, g)
    V = np.stack([_det_state(norb, *S.det(i), cre) for i in range(S.ndet)], axis=1)
    Hproj = V.T @ (Hb @ V)
    Ho = S.hmat()
    return np.abs(Ho - Hproj).max(), np.abs(Hproj).max()


@pytest.mark.parametrize("norb,na,nb,seed", [(4, 2, 2, 0), (4, 3, 1, 1), (5, 2, 3, 2), (5, 1, 1, 3),
                                             (4, 0, 2, 4), (3, 3, 2, 5), (5, 3, 3, 6)])
def test_slater_condon_matches_eq6_brute_force(norb, na, nb, seed):
    err, scale = _oracle_vs_brute(norb, na, nb, seed)
    assert scale > 0.1
    assert err < 1e-12 * max(1.0, scale)


def test_slater_condon_matches_brute_force_gas():
    # two GAS spaces (2 + 3 orbitals), 4 electrons, at most one hole in space 1
    err, scale = _oracle_vs_brute(5, 2, 2, 7, gas=([2, 3], [3, 4], [4, 4]))
    assert err < 1e-12 * max(1.0, scale)


def test_brute_force_detects_planted_sign_error():
    """The brute-force pin is sensitive: flipping one exchange sign in a copy of
    the Slater-Condon diagonal formula breaks agreement."""
    norb, na, nb = 4, 2, 2
    h, g = si.integrals(norb, 8, 11)
    S = oracle.Space(norb, na, nb, h, g)
    Hb, cre = _brute_h(norb, h, g)
    i = 5
    v = _det_state(norb, *S.det(i), cre)
    ref = v @ (Hb @ v)
    ia, ib = S.det(i)
    occa = [p for p in range(norb) if (ia >> p) & 1]
    occb = [p for p in range(norb) if (ib >> p) & 1]
    e_wrong = sum(h[p, p] for p in occa + occb)
    for occ in (occa, occb):
        for p in occ:
            for q in occ:
                e_wrong += 0.5 * (g[p, p, q, q] + g[p, q, q, p])   # planted: + exchange
    for p in occa:
        for q in occb:
            e_wrong += g[p, p, q, q]
    assert abs(S.h_elem(i, i) - ref) < 1e-12
    assert abs(e_wrong - ref) > 1e-3


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t,U", [(1.0, 3.0), (0.7, 0.0), (1.3, 5.5)])
def test_two_site_hubbard(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0] = g[1, 1, 1, 1] = U
    S = oracle.Space(2, 1, 1, h, g)
    w = np.sort(np.linalg.eigvalsh(S.hmat()))
    r = math.sqrt(U * U + 16 * t * t)
    ref = np.sort([(U - r) / 2, 0.0, U, (U + r) / 2])
    assert np.allclose(w, ref, atol=1e-12)


@pytest.mark.parametrize("norb,na,nb", [(5, 2, 2), (6, 3, 2), (5, 1, 4)])
def test_non_interacting_spectrum(norb, na, nb):
    h, _ = si.integrals(norb, 4, 21)
    g = np.zeros((norb,) * 4)
    S = oracle.Space(norb, na, nb, h, g)
    w = np.sort(np.linalg.eigvalsh(S.hmat()))
    eps = np.linalg.eigvalsh(h)
    sums = sorted(sum(eps[list(a)]) + sum(eps[list(b)])
                  for a in itertools.combinations(range(norb), na)
                  for b in itertools.combinations(range(norb), nb))
    assert np.allclose(w, sums, atol=1e-12)


def test_non_interacting_ground_state_davidson():
    norb, na, nb = 9, 3, 4
    h, _ = si.integrals(norb, 4, 22)
    S = oracle.Space(norb, na, nb, h, np.zeros((norb,) * 4))
    e, _, info = oracle.davidson(S, 1, tol=1e-12)
    eps = np.linalg.eigvalsh(h)
    assert abs(e[0] - (eps[:na].sum() + eps[:nb].sum())) < 1e-9


# ---------------------------------------------------------------------------
# symmetries and invariants
# ---------------------------------------------------------------------------
def _s2_matrix(S):
    """S^2 = S_z^2 + S_z + S_- S_+ in the oracle basis, from bit operations."""
    n = S.norb
    dets = [S.det(i) for i in range(S.ndet)]
    index = {d: i for i, d in enumerate(dets)}
    sz = 0.5 * (S.nalpha - S.nbeta)
    M = np.zeros((S.ndet, S.ndet))
    M[np.arange(S.ndet), np.arange(S.ndet)] = sz * sz + sz

    def apply_op(ops, a, b, sign=1.0):
        # ops: list of (kind, spin, orb) applied right to left; JW order alpha 0..n-1, beta n..2n-1
        bits = a | (b << n)
        for kind, spin, p in reversed(ops):
            so = p + spin * n
            occ = (bits >> so) & 1
            if kind == "c" and occ or kind == "a" and not occ:
                return None
            if bin(bits & ((1 << so) - 1)).count("1") % 2:
                sign = -sign
            bits ^= 1 << so
        return bits & ((1 << n) - 1), bits >> n, sign

    for j, (a, b) in enumerate(dets):
        # S_- S_+ = sum_pq a+_qb a_qa a+_pa a_pb
        for p in range(n):
            for q in range(n):
                r = apply_op([("c", 1, q), ("a", 0, q), ("c", 0, p), ("a", 1, p)], a, b)
                if r is None:
                    continue
                i = index.get((r[0], r[1]))
                if i is not None:
                    M[i, j] += r[2]
    return M


@pytest.mark.parametrize("norb,na,nb", [(5, 2, 2), (5, 3, 2), (4, 2, 1)])
def test_h_commutes_with_s2(norb, na, nb):
    h, g = si.integrals(norb, 10, 31)
    S = oracle.Space(norb, na, nb, h, g)
    H = S.hmat()
    S2 = _s2_matrix(S)
    assert np.abs(S2 - S2.T).max() < 1e-12
    assert np.abs(H @ S2 - S2 @ H).max() < 1e-11
    # and S^2 eigenvalues are s(s+1)
    w = np.linalg.eigvalsh(S2)
    s = (-1 + np.sqrt(1 + 4 * w)) / 2
    assert np.allclose(2 * s, np.round(2 * s), atol=1e-9)


def test_h_symmetric_and_sigma_is_dense_product():
    h, g = si.integrals(6, 12, 0)
    S = oracle.Space(6, 3, 2, h, g)
    H = S.hmat()
    assert np.abs(H - H.T).max() < 1e-13
    C = si.ci_vector(S.ndet, 3)
    assert np.abs(S.sigma(C) - H @ C).max() < 1e-12
    rows = np.array([0, 7, S.ndet - 1, 33])
    assert np.abs(S.sigma_rows(rows, C) - (H @ C)[rows]).max() < 1e-12
    assert np.abs(S.hdiag() - np.diag(H)).max() < 1e-13


def test_sigma_symmetry_and_transposition():
    h, g = si.integrals(7, 14, 5)
    S = oracle.Space(7, 3, 3, h, g)
    n = int(round(math.sqrt(S.ndet)))
    c1, c2 = si.ci_vector(S.ndet, 1), si.ci_vector(S.ndet, 2)
    s1, s2 = S.sigma(c1), S.sigma(c2)
    assert abs(c1 @ s2 - c2 @ s1) < 1e-12
    # alpha <-> beta transposition (n_alpha = n_beta, CAS): sigma(C^T) = sigma(C)^T
    M = c1.reshape(n, n)
    sT = S.sigma(M.T.copy().reshape(-1)).reshape(n, n)
    assert np.abs(sT - s1.reshape(n, n).T).max() < 1e-12


def _embed(Sg, Sc, cg):
    """GAS vector -> CAS vector (zeros outside the GAS space) and index map."""
    idx = np.array([Sc.address(*Sg.det(i)) for i in range(Sg.ndet)])
    assert (idx >= 0).all()
    cc = np.zeros(Sc.ndet)
    cc[idx] = cg
    return cc, idx


def test_unrestricted_gas_equals_cas():
    norb, na, nb = 6, 3, 3
    h, g = si.integrals(norb, 12, 8)
    Sc = oracle.Space(norb, na, nb, h, g)
    Sg = oracle.Space(norb, na, nb, h, g, gas=([2, 2, 2], [0, 0, 6], [6, 6, 6]))
    assert Sg.ndet == Sc.ndet
    cg = si.ci_vector(Sg.ndet, 4)
    cc, idx = _embed(Sg, Sc, cg)
    assert np.abs(Sg.sigma(cg) - Sc.sigma(cc)[idx]).max() < 1e-12


def test_restricted_gas_is_projected_cas():
    norb, na, nb = 7, 3, 3
    h, g = si.integrals(norb, 14, 9)
    Sc = oracle.Space(norb, na, nb, h, g)
    Sg = oracle.Space(norb, na, nb, h, g, gas=([2, 3, 2], [3, 5, 6], [4, 6, 6]))
    assert 0 < Sg.ndet < Sc.ndet
    cg = si.ci_vector(Sg.ndet, 5)
    cc, idx = _embed(Sg, Sc, cg)
    assert np.abs(Sg.sigma(cg) - Sc.sigma(cc)[idx]).max() < 1e-12


# ---------------------------------------------------------------------------
# counting and ordering
# ---------------------------------------------------------------------------
def _golden_counts():
    out = {}
    with open(os.path.join(GOLDEN, "paper_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = int(val)
    return out


def test_paper_determinant_counts():
    gc = _golden_counts()
    assert math.comb(22, 11) ** 2 == gc["cas22_full"]
    assert math.comb(24, 12) ** 2 == gc["cas24_full"]
    # M_S = 0 combinations: pairs {I_a, I_b} counted once, diagonal ones once
    assert (gc["cas20_d2h"] + math.comb(20, 10)) // 2 == gc["cas20_d2h_combinations"]
    assert 6 ** 4 == gc["loop_types_6gas"] and 8 ** 4 == gc["loop_types_8gas"]
    for norb, na, nb in [(6, 3, 3), (8, 5, 2), (10, 0, 4)]:
        h, g = np.zeros((norb, norb)), np.zeros((norb,) * 4)
        assert oracle.Space(norb, na, nb, h, g).ndet == math.comb(norb, na) * math.comb(norb, nb)


def _contract_order(norb, na, nb, gas):
    """Independent itertools implementation of the determinant ordering contract."""
    gn, gmin, gmax = gas
    first = np.cumsum([0] + list(gn))

    def occ(bits):
        return tuple(bin(bits & (((1 << gn[k]) - 1) << first[k])).count("1") for k in range(len(gn)))

    def allowed(ta, tb):
        cum = 0
        for k in range(len(gn)):
            cum += ta[k] + tb[k]
            if not gmin[k] <= cum <= gmax[k]:
                return False
        return True

    strs = []
    for ne in (na, nb):
        s = sorted(sum(1 << p for p in c) for c in itertools.combinations(range(norb), ne))
        strs.append(s)
    types = [sorted({occ(x) for x in s}) for s in strs]
    order = []
    for ta in types[0]:
        for tb in types[1]:
            if not allowed(ta, tb):
                continue
            A = [x for x in strs[0] if occ(x) == ta]
            B = [x for x in strs[1] if occ(x) == tb]
            order += [(a, b) for a in A for b in B]
    return order


def test_ordering_contract_gas():
    gas = ([2, 3, 2], [3, 5, 6], [4, 6, 6])
    h, g = np.zeros((7, 7)), np.zeros((7,) * 4)
    S = oracle.Space(7, 3, 3, h, g, gas=gas)
    ref = _contract_order(7, 3, 3, gas)
    assert S.ndet == len(ref)
    assert [S.det(i) for i in range(S.ndet)] == ref


def test_gas20_count_independent():
    """GAS 20e/20o, spaces 6/8/6, cumulative bounds [10,12],[18,20],[20,20]:
    count from an independent per-type tally of itertools strings."""
    w = si.WORKLOADS["gas20"]
    gn, gmin, gmax = w["gas"]
    cnt = {}
    for c in itertools.combinations(range(20), 10):
        t = (sum(1 for p in c if p < 6), sum(1 for p in c if 6 <= p < 14), sum(1 for p in c if p >= 14))
        cnt[t] = cnt.get(t, 0) + 1
    total = 0
    for ta, na_ in cnt.items():
        for tb, nb_ in cnt.items():
            c1 = ta[0] + tb[0]
            c2 = c1 + ta[1] + tb[1]
            if gmin[0] <= c1 <= gmax[0] and gmin[1] <= c2 <= gmax[1]:
                total += na_ * nb_
    h, g = np.zeros((20, 20)), np.zeros((20,) * 4)
    S = oracle.Space(20, 10, 10, h, g, gas=w["gas"])
    assert S.ndet == total
    ta, tb, off = S.blocks()
    assert len(ta) == 36


# ---------------------------------------------------------------------------
# Davidson
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("norb,na,nb,nroots", [(6, 3, 3, 1), (6, 3, 3, 3), (7, 4, 2, 2)])
def test_davidson_matches_dense(norb, na, nb, nroots):
    h, g = si.integrals(norb, 2 * norb, 0)
    S = oracle.Space(norb, na, nb, h, g)
    w = np.linalg.eigvalsh(S.hmat())
    e, X, info = oracle.davidson(S, nroots, tol=1e-11, max_space=12)
    assert info["converged"]
    assert np.allclose(e, w[:nroots], atol=1e-9)
    # residual certificate: |theta - lambda| <= ||r||
    for k in range(nroots):
        r = np.linalg.norm(S.sigma(X[k]) - e[k] * X[k])
        assert np.min(np.abs(w - e[k])) <= r + 1e-12


def test_davidson_cas8_vs_dense():
    h, g = si.integrals(8, 16, 0)
    S = oracle.Space(8, 4, 4, h, g)
    w = np.linalg.eigvalsh(S.hmat())
    e, _, info = oracle.davidson(S, 2, tol=1e-10)
    assert np.allclose(e, w[:2], atol=1e-8)


# ---------------------------------------------------------------------------
# M_S = 0 sectors (Sec. 3.1, Sec. 3.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("norb,ne,seed", [(5, 2, 3), (4, 2, 8), (6, 3, 1)])
def test_parity_sectors_split_the_spectrum(norb, ne, seed):
    """The two sectors are orthogonal complements invariant under H (which
    commutes with alpha <-> beta exchange), so their spectra together are the
    whole spectrum."""
    h, g = si.integrals(norb, 2 * norb, seed)
    S = oracle.Space(norb, ne, ne, h, g)
    n = int(round(math.sqrt(S.ndet)))
    Qe, Qo = oracle.parity_basis(n, 1), oracle.parity_basis(n, -1)
    assert Qe.shape[0] == n * (n + 1) // 2 and Qo.shape[0] == n * (n - 1) // 2
    Q = np.vstack([Qe, Qo])
    assert np.abs(Q @ Q.T - np.eye(S.ndet)).max() < 1e-14
    H = S.hmat()
    assert np.abs(Qe @ H @ Qo.T).max() < 1e-12
    both = np.sort(np.concatenate([oracle.parity_spectrum(S, 1), oracle.parity_spectrum(S, -1)]))
    assert np.allclose(both, np.linalg.eigvalsh(H), atol=1e-11)


@pytest.mark.parametrize("norb,ne", [(5, 2), (4, 2), (4, 1)])
def test_parity_sector_total_spin(norb, ne):
    """With the determinant order alpha string before beta string, the
    symmetric sector holds exactly the even total spins S and the
    antisymmetric one the odd S."""
    h, g = si.integrals(norb, 2 * norb, 4)
    S = oracle.Space(norb, ne, ne, h, g)
    n = int(round(math.sqrt(S.ndet)))
    S2 = _s2_matrix(S)
    for parity in (1, -1):
        Q = oracle.parity_basis(n, parity)
        w = np.linalg.eigvalsh(Q @ S2 @ Q.T)
        s = np.round((-1 + np.sqrt(1 + 4 * w)) / 2).astype(int)
        assert np.allclose(s * (s + 1), w, atol=1e-9)
        assert np.all(s % 2 == (0 if parity > 0 else 1)), (parity, sorted(set(s)))


@pytest.mark.parametrize("norb,ne,seed", [(5, 2, 3), (4, 2, 8)])
def test_parity_basis_dets_is_the_one_block_basis(norb, ne, seed):
    """For one-block spaces the sector basis built from the determinant list is
    the one-block basis row for row."""
    h, g = si.integrals(norb, 2 * norb, seed)
    S = oracle.Space(norb, ne, ne, h, g)
    n = int(round(math.sqrt(S.ndet)))
    for parity in (1, -1):
        assert np.array_equal(oracle.parity_basis_dets(S, parity), oracle.parity_basis(n, parity))


@pytest.mark.parametrize("norb,ne,gas,orbsym,target", [
    (7, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]), None, 0),
    (6, 3, ([2, 2, 2], [0, 0, 6], [6, 6, 6]), None, 0),
    (6, 3, None, [0, 1, 2, 3, 0, 1], 0),
    (6, 2, None, [0, 1, 2, 3, 0, 1], 3),
])
def test_parity_sectors_of_blocked_spaces(norb, ne, gas, orbsym, target):
    """GAS and point-group spaces with n_alpha = n_beta: the two sector bases
    together are an orthonormal basis of the space, every basis vector is even
    or odd under the exchange of the alpha and beta strings, H couples no even
    vector to an odd one, and the two sector spectra together are the spectrum
    of H."""
    h, g = si.integrals(norb, 2 * norb, 6, orbsym=orbsym)
    S = oracle.Space(norb, ne, ne, h, g, gas=gas, orbsym=orbsym, target=target)
    d = S.dets()
    swap = np.array([S.address(int(b), int(a)) for a, b in d])
    Qe, Qo = oracle.parity_basis_dets(S, 1), oracle.parity_basis_dets(S, -1)
    Q = np.vstack([Qe, Qo])
    assert Q.shape[0] == S.ndet
    assert np.abs(Q @ Q.T - np.eye(S.ndet)).max() < 1e-14
    assert np.array_equal(Qe[:, swap], Qe) and np.array_equal(Qo[:, swap], -Qo)
    H = S.hmat()
    assert np.abs(Qe @ H @ Qo.T).max() < 1e-12
    both = np.sort(np.concatenate([oracle.parity_spectrum_dets(S, 1), oracle.parity_spectrum_dets(S, -1)]))
    assert np.allclose(both, np.linalg.eigvalsh(H), atol=1e-11)


@pytest.mark.parametrize("t,U", [(1.0, 3.0), (1.3, 5.5)])
def test_parity_two_site_hubbard(t, U):
    """Two electrons on two sites: the three singlets (U -+ r)/2 and U are the
    symmetric sector, the M_S = 0 triplet (energy 0) the antisymmetric one."""
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0] = g[1, 1, 1, 1] = U
    S = oracle.Space(2, 1, 1, h, g)
    r = math.sqrt(U * U + 16 * t * t)
    assert np.allclose(oracle.parity_spectrum(S, 1), sorted([(U - r) / 2, U, (U + r) / 2]), atol=1e-12)
    assert np.allclose(oracle.parity_spectrum(S, -1), [0.0], atol=1e-12)


# ---------------------------------------------------------------------------
# density matrices (plain operator application)
# ---------------------------------------------------------------------------
RDM_CASES = [(5, 2, 2, None), (6, 3, 2, None), (5, 1, 3, None), (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]))]


@pytest.mark.parametrize("case", RDM_CASES, ids=[f"n{c[0]}a{c[1]}b{c[2]}" + ("gas" if c[3] else "") for c in RDM_CASES])
def test_rdm_energy_traces_and_symmetries(case):
    """sum h gamma + 1/2 sum (pq|rs) Gamma = <C|H|C>/<C|C> with H C from the
    Slater-Condon sigma (independent code); traces N and N(N-1); partial trace
    (N-1) gamma; Gamma_pqrs = Gamma_rspq = Gamma_qpsr."""
    norb, na, nb, gas = case
    h, g = si.integrals(norb, 2 * norb, 13)
    S = oracle.Space(norb, na, nb, h, g, gas=gas)
    C = si.ci_vector(S.ndet, 5)
    g1, g2 = S.rdm(C)
    N = na + nb
    e_rdm = np.einsum("pq,pq", h, g1) + 0.5 * np.einsum("pqrs,pqrs", g, g2)
    e_sig = C @ S.sigma(C) / (C @ C)
    assert abs(e_rdm - e_sig) < 1e-12 * max(1.0, abs(e_sig))
    assert abs(np.trace(g1) - N) < 1e-12
    assert abs(np.einsum("pprr", g2) - N * (N - 1)) < 1e-11
    assert np.abs(np.einsum("pqrr->pq", g2) - (N - 1) * g1).max() < 1e-12
    assert np.abs(g1 - g1.T).max() < 1e-13
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() < 1e-13
    assert np.abs(g2 - g2.transpose(1, 0, 3, 2)).max() < 1e-13


def test_rdm_single_determinant_closed_form():
    """One determinant: gamma = diag(n_a + n_b) and
    Gamma_pqrs = d_pq d_rs (N_p N_r - d_pr N_p) - d_ps d_qr (sum_s n_ps n_qs - d_pq N_p)."""
    norb, na, nb = 5, 3, 2
    h, g = si.integrals(norb, 10, 2)
    S = oracle.Space(norb, na, nb, h, g)
    i = 7
    C = np.zeros(S.ndet)
    C[i] = -2.0
    ia, ib = S.det(i)
    na_ = np.array([(ia >> p) & 1 for p in range(norb)], float)
    nb_ = np.array([(ib >> p) & 1 for p in range(norb)], float)
    Np = na_ + nb_
    d = np.eye(norb)
    same = np.outer(na_, na_) + np.outer(nb_, nb_)
    want2 = (np.einsum("pq,rs,p,r->pqrs", d, d, Np, Np) - np.einsum("pq,rs,pr,p->pqrs", d, d, d, Np)
             - np.einsum("ps,qr,pq->pqrs", d, d, same) + np.einsum("ps,qr,pq,p->pqrs", d, d, d, Np))
    g1, g2 = S.rdm(C)
    assert np.abs(g1 - np.diag(Np)).max() < 1e-14
    assert np.abs(g2 - want2).max() < 1e-14


def test_cas66_recipe_values():
    """The CAS(6,6) workload under the seeded recipe against values recorded
    independently when the workloads were defined (tests/golden/cas66_recipe.txt):
    diag(h) to the 6 printed decimals, (00|00), the lowest diagonal element and
    its index, and the four lowest eigenvalues of the oracle's dense H."""
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "cas66_recipe.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, v = ln.split()
                vals[k] = float(v)
    h, g = si.integrals(6, 12, 0)
    for p in range(6):
        assert abs(h[p, p] - vals[f"h{p}{p}"]) <= 5e-7
    assert abs(g[0, 0, 0, 0] - vals["eri0000"]) <= 1e-12
    sp = oracle.Space(6, 3, 3, h, g)
    d = sp.hdiag()
    assert int(np.argmin(d)) == int(vals["argmin_hdiag"])
    assert abs(d.min() - vals["min_hdiag"]) <= 1e-11
    w = np.linalg.eigvalsh(sp.hmat())
    for k in range(4):
        assert abs(w[k] - vals[f"E{k}"]) <= 1e-11, (k, w[k])


# ---- spatial symmetry (the S of the TTSS blocks, Sec. 3.1 Eq. 9; D2h spaces, Sec. 4-5) ----

SYM_CASES = [
    (6, 3, 3, [0, 1, 2, 3, 0, 1], None),
    (7, 3, 2, [0, 1, 2, 3, 4, 5, 6], None),
    (8, 4, 4, [p % 8 for p in range(8)], None),
    (7, 3, 3, [0, 1, 1, 2, 3, 0, 5], ([2, 3, 2], [3, 5, 6], [4, 6, 6])),
]


def _sym_tally(norb, na, nb, orbsym, target, gas):
    """Independent count and order of the symmetric space: itertools strings,
    irreps by XOR, GAS bounds, types (counts per space, irrep) sorted."""
    gn, mn, mx = gas if gas else ([norb], [na + nb], [na + nb])
    first = np.concatenate([[0], np.cumsum(gn)[:-1]])

    def strings(ne):
        out = []
        for occ in itertools.combinations(range(norb), ne):
            x = sum(1 << p for p in occ)
            cnt = tuple(sum(1 for p in occ if first[g] <= p < first[g] + gn[g]) for g in range(len(gn)))
            irr = 0
            for p in occ:
                irr ^= orbsym[p]
            out.append((cnt + (irr,), x))
        return out

    def ok(ta, tb):
        c = 0
        for g in range(len(gn)):
            c += ta[g] + tb[g]
            if c < mn[g] or c > mx[g]:
                return False
        return (ta[-1] ^ tb[-1]) == target

    A, B = strings(na), strings(nb)
    ta_all = sorted({t for t, _ in A})
    tb_all = sorted({t for t, _ in B})
    ta_k = [t for t in ta_all if any(ok(t, u) for u in tb_all)]
    tb_k = [u for u in tb_all if any(ok(t, u) for t in ta_all)]
    dets = []
    for t in ta_k:
        for u in tb_k:
            if ok(t, u):
                sa = sorted(x for tt, x in A if tt == t)
                sb = sorted(x for tt, x in B if tt == u)
                dets += [(a, b) for a in sa for b in sb]
    return dets


@pytest.mark.parametrize("case", SYM_CASES, ids=lambda c: f"n{c[0]}a{c[1]}b{c[2]}" + ("gas" if c[4] else ""))
def test_symmetric_space_order_and_counts(case):
    norb, na, nb, orbsym, gas = case
    h, g = si.integrals(norb, 2 * norb, 1, orbsym=orbsym)
    total = 0
    for target in range(8):
        want = _sym_tally(norb, na, nb, orbsym, target, gas)
        sp = oracle.Space(norb, na, nb, h, g, gas=gas, orbsym=orbsym, target=target)
        assert sp.ndet == len(want)
        if sp.ndet:
            got = [tuple(int(v) for v in d) for d in sp.dets()]
            assert got == want
        total += sp.ndet
    assert total == oracle.Space(norb, na, nb, h, g, gas=gas).ndet


def test_symmetric_integrals_recipe():
    orbsym = [p % 8 for p in range(10)]
    h, g = si.integrals(10, 20, 3, orbsym=orbsym)
    s = np.array(orbsym)
    assert np.all(h[(s[:, None] != s[None, :])] == 0)
    x = s[:, None, None, None] ^ s[None, :, None, None] ^ s[None, None, :, None] ^ s[None, None, None, :]
    assert np.all(g[x != 0] == 0)
    assert np.abs(g[x == 0]).max() > 1e-3
    assert np.allclose(g, g.transpose(1, 0, 2, 3)) and np.allclose(g, g.transpose(2, 3, 0, 1))
    assert np.linalg.eigvalsh(g.reshape(100, 100)).min() > -1e-12
    # the draws before the shaping are those of the unsymmetric recipe
    h0, _ = si.integrals(10, 20, 3)
    assert np.array_equal(np.diag(h), np.diag(h0))


@pytest.mark.parametrize("case", SYM_CASES[:3], ids=lambda c: f"n{c[0]}a{c[1]}b{c[2]}")
def test_symmetry_blocks_split_the_spectrum(case):
    """H with point-group integrals has no element between determinants of
    different total irrep: the spectra of the eight symmetric spaces together
    are the spectrum of the whole space (dense eigh), and sigma of a vector
    of one symmetric space, embedded in the whole space, vanishes outside it
    and equals that space's own sigma inside."""
    norb, na, nb, orbsym, gas = case
    h, g = si.integrals(norb, 2 * norb, 2, orbsym=orbsym)
    full = oracle.Space(norb, na, nb, h, g, gas=gas)
    w_full = np.linalg.eigvalsh(full.hmat())
    parts = []
    for target in range(8):
        sp = oracle.Space(norb, na, nb, h, g, gas=gas, orbsym=orbsym, target=target)
        if sp.ndet == 0:
            continue
        parts.append(np.linalg.eigvalsh(sp.hmat()))
        c = si.ci_vector(sp.ndet, target)
        idx = np.array([full.address(int(a), int(b)) for a, b in sp.dets()])
        C = np.zeros(full.ndet)
        C[idx] = c
        s_full = full.sigma(C)
        s_sym = sp.sigma(c)
        assert np.allclose(s_full[idx], s_sym, atol=1e-12)
        mask = np.ones(full.ndet, bool)
        mask[idx] = False
        assert np.abs(s_full[mask]).max() <= 1e-12
    assert np.allclose(np.sort(np.concatenate(parts)), w_full, atol=1e-10)
