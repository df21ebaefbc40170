"""The direction of the T1 transformation, pinned in second quantisation.

The oracle transforms every one-index object as h -> (1 - t) h (1 + t), with
t[no+a][i] = t^a_i (the T1-transformed Hamiltonian exp(-T1) H exp(T1) of Sec.
Theory).  The similarity and block checks elsewhere would pass unchanged under
the opposite direction (1 + t) h (1 - t), i.e. exp(T1) H exp(-T1).  Here the
transformation is computed without the oracle: on the Fock space of a tiny
system (two occupied and two virtual spatial orbitals, eight spin orbitals,
dimension 256) the singlet excitation operators E_pq = sum_sigma a+_{p sigma}
a_{q sigma} are built as matrices (Jordan-Wigner), T1 = sum_ai t^a_i E_ai is
exponentiated exactly (it is nilpotent), and exp(-T1) H exp(T1) is compared, as
an operator, with the operator built from the oracle's transformed integrals.
"""
import numpy as np
import pytest

from oracle import cc3_oracle as O

NO, NV = 2, 2
NMO = NO + NV
NMODE = 2 * NMO  # spin orbitals, mode 2p + sigma


def _annihilators():
    z = np.diag([1.0, -1.0])
    low = np.array([[0.0, 1.0], [0.0, 0.0]])  # |1> -> |0>
    eye = np.eye(2)
    ops = []
    for m in range(NMODE):
        mats = [z] * m + [low] + [eye] * (NMODE - m - 1)
        a = mats[0]
        for x in mats[1:]:
            a = np.kron(a, x)
        ops.append(a)
    return ops


A = _annihilators()
E = [[sum(A[2 * p + s].T @ A[2 * q + s] for s in range(2)) for q in range(NMO)]
     for p in range(NMO)]


def one_body(h):
    return sum(h[p, q] * E[p][q] for p in range(NMO) for q in range(NMO))


def two_body(g):
    """sum_pqrs g_pqrs E_pq E_rs."""
    out = np.zeros_like(E[0][0])
    for p in range(NMO):
        for q in range(NMO):
            inner = sum(g[p, q, r, s] * E[r][s] for r in range(NMO) for s in range(NMO))
            out = out + E[p][q] @ inner
    return out


def expm_nilpotent(x):
    """exp(x) for nilpotent x: the finite power series (checked to terminate)."""
    out = np.eye(x.shape[0])
    term = np.eye(x.shape[0])
    for n in range(1, 40):
        term = term @ x / n
        if not term.any():
            return out
        out = out + term
    raise AssertionError("T1 is not nilpotent")


@pytest.fixture(scope="module")
def system():
    rng = np.random.default_rng(20070108)
    t1 = rng.normal(0.0, 0.3, size=(NO, NV))
    T1 = sum(t1[i, a] * E[NO + a][i] for i in range(NO) for a in range(NV))
    return t1, expm_nilpotent(-T1), expm_nilpotent(T1)


def test_anticommutation_of_the_construction():
    for m in range(NMODE):
        for n in range(NMODE):
            ac = A[m] @ A[n].T + A[n].T @ A[m]
            assert np.array_equal(ac, np.eye(256) * (m == n))


def test_one_body_transformation_direction(system):
    t1, em, ep = system
    rng = np.random.default_rng(3)
    h = rng.normal(size=(NMO, NMO))  # any one-index object, not necessarily symmetric
    ref = em @ one_body(h) @ ep
    got = one_body(O.t1_transform(h[None], t1)[0])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    # the opposite direction, exp(T1) H exp(-T1) = (1 + t) h (1 - t), is a different operator
    t = np.zeros((NMO, NMO))
    t[NO:, :NO] = t1.T
    wrong = one_body((np.eye(NMO) + t) @ h @ (np.eye(NMO) - t))
    assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()


def test_two_body_from_transformed_cholesky_vectors(system):
    """exp(-T1) (sum_J (L^J . E)^2) exp(T1) equals the operator of
    g~_pqrs = sum_J Lt^J_pq Lt^J_rs with the oracle's Lt, and the oracle's integral
    blocks are the corresponding slices of g~ in the paper's index order."""
    t1, em, ep = system
    rng = np.random.default_rng(4)
    L = rng.normal(0.0, 0.3, size=(3, NMO, NMO))
    L = L + L.transpose(0, 2, 1)
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    ref = em @ two_body(g) @ ep
    Lt = O.t1_transform(L, t1)
    gt = np.einsum("Jpq,Jrs->pqrs", Lt, Lt)
    got = two_body(gt)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    blk = O.IntegralBlocks(Lt, NO, full=True)
    o, v = slice(0, NO), slice(NO, NMO)
    assert np.allclose(blk.full_vvvo(), gt[v, v, v, o], rtol=0, atol=1e-14)   # g_{bdck}
    assert np.allclose(blk.g_oovo, gt[o, o, v, o], rtol=0, atol=1e-14)       # g_{ljck}
    assert np.allclose(blk.g_ovov, gt[o, v, o, v], rtol=0, atol=1e-14)       # g_{jbkc}
    assert np.allclose(blk.g_ooov, gt[o, o, o, v], rtol=0, atol=1e-14)       # g_{jlkc}
    assert np.allclose(blk.full_vvov(), gt[v, v, o, v], rtol=0, atol=1e-14)  # g_{dbkc}
    # the ov block of the Cholesky vectors is unchanged by the transformation
    assert np.array_equal(Lt[:, o, v], L[:, o, v])
