"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these retypes the oracle's formula: each compares it with an
independent evaluation (brute force over the full T3 tensor with a full
four-index T1 transformation), a closed form (the closed-shell [T] energy
functional, the S3 spectrum of the contravariant combination), an invariant
(the permutational symmetry of t3, similarity invariants of the T1
transformation, homogeneity degrees) or the paper's own printed timings.
"""
import json
import os
from math import comb

import numpy as np
import pytest

from oracle import cc3_oracle as O
from oracle import bruteforce as B
from oracle.bruteforce import residual_bruteforce, transformed_hamiltonian
from paper_2007_01088_amd.synth import make_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _blocks(d):
    Lt = O.t1_transform(d["L"], d["t1"])
    return O.IntegralBlocks(Lt, d["no"], full=True), O.fock_ov(d["L"], d["t1"])


@pytest.mark.parametrize("no,nv,nJ,t1z", [(3, 4, 10, True), (3, 4, 10, False), (4, 5, 12, False),
                                          (4, 6, 12, True), (4, 6, 14, False), (4, 20, 30, False),
                                          (5, 7, 15, False), (2, 3, 8, False)])
def test_loop_oracle_equals_bruteforce(no, nv, nJ, t1z):
    """Algorithm 1's restricted loop reaches the full-T3 definition (Sec. Implementation)."""
    d = make_inputs(no, nv, nJ, t1_zero=t1z)
    o1, o2 = O.triples_residual(d["eps"], d["L"], d["t1"], d["t2"])
    b1, b2, _ = residual_bruteforce(d["eps"], d["L"], d["t1"], d["t2"])
    assert np.abs(b2).max() > 1e-6
    assert rel(o1, b1) < 1e-13
    assert rel(o2, b2) < 1e-13


def test_t3_permutational_symmetry():
    """tau^{abc}_{ijk} = tau^{bac}_{jik} = tau^{cba}_{kji} = tau^{acb}_{ikj} = tau^{cab}_{kij} = tau^{bca}_{jki}."""
    d = make_inputs(5, 7, 15)
    blk, _ = _blocks(d)
    eps, t2 = d["eps"], d["t2"]
    i, j, k = 4, 2, 1
    t = O.t3_amplitudes(i, j, k, eps, t2, blk)
    assert np.abs(t).max() > 1e-6
    pairs = [((j, i, k), "bac"), ((k, j, i), "cba"), ((i, k, j), "acb"),
             ((k, i, j), "cab"), ((j, k, i), "bca")]
    for (p, q, r), lab in pairs:
        other = O.t3_amplitudes(p, q, r, eps, t2, blk)
        # tau_{pqr} evaluated at the permuted virtual labels equals tau_{ijk}[a,b,c]
        assert rel(np.einsum(lab + "->abc", other), t) < 1e-13, (p, q, r)
    # and the occupied-permutation views used by the restricted loop agree with a direct build
    tt = O.contravariant(t)
    for (p, q, r), U in O.occupied_permutations(i, j, k, tt):
        direct = O.contravariant(O.t3_amplitudes(p, q, r, eps, t2, blk))
        assert rel(U, direct) < 1e-13, (p, q, r)


def test_contravariant_s3_spectrum():
    """4e - 2(sum of transpositions) + (sum of 3-cycles) acts on S3 isotypic parts as 0, 3, 12."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(6, 6, 6))
    perms = ["abc", "acb", "bac", "cba", "bca", "cab"]
    sign = [1, -1, -1, -1, 1, 1]
    sym = sum(np.einsum(p + "->abc", x) for p in perms)
    anti = sum(s * np.einsum(p + "->abc", x) for p, s in zip(perms, sign))
    std = x - sym / 6.0 - anti / 6.0
    assert np.abs(O.contravariant(sym)).max() < 1e-12
    assert rel(O.contravariant(anti), 12.0 * anti) < 1e-13
    assert rel(O.contravariant(std), 3.0 * std) < 1e-13


def test_t_energy_functional_at_t1_zero():
    """With t1 = 0, sum (2t^{ab}_{ij} - t^{ba}_{ij}) Omega^{ab}_{ij} equals the closed-shell
    fourth-order triples energy 1/3 sum (4X^{abc} + X^{bca} + X^{cab})(X^{abc} - X^{cba}) / D,
    D = e_i + e_j + e_k - e_a - e_b - e_c, X = P W.  Pins every index order of the Omega
    contractions and the 1/3 P normalisation of the back-transformation."""
    d = make_inputs(5, 8, 16, t1_zero=True)
    eps, L, t2 = d["eps"], d["L"], d["t2"]
    no, nv = d["no"], d["nv"]
    _, o2 = O.triples_residual(eps, L, d["t1"], t2)
    lhs = np.sum((2.0 * t2 - t2.transpose(0, 1, 3, 2)) * o2)
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    o, v = slice(0, no), slice(no, None)
    W = (np.einsum("ijad,bdck->ijkabc", t2, g[v, v, v, o])
         - np.einsum("ilab,ljck->ijkabc", t2, g[o, o, v, o]))
    X = (W + np.einsum("jikbac->ijkabc", W) + np.einsum("kjicba->ijkabc", W)
         + np.einsum("ikjacb->ijkabc", W) + np.einsum("jkibca->ijkabc", W)
         + np.einsum("kijcab->ijkabc", W))
    eo, ev = eps[:no], eps[no:]
    D = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
         + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
         - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    Xbca = np.einsum("ijkbca->ijkabc", X)
    Xcab = np.einsum("ijkcab->ijkabc", X)
    Xcba = np.einsum("ijkcba->ijkabc", X)
    rhs = np.sum((4.0 * X + Xbca + Xcab) * (X - Xcba) / D) / 3.0
    assert rhs < 0.0
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_homogeneity_and_symmetry():
    """Omega(t2 = 0) = 0; linear in t2; Omega(s*eps) = Omega/s; Omega(s*L) = s^4 Omega;
    Omega^{ab}_{ij} = Omega^{ba}_{ji}."""
    d = make_inputs(4, 6, 12)
    eps, L, t1, t2 = d["eps"], d["L"], d["t1"], d["t2"]
    o1, o2 = O.triples_residual(eps, L, t1, t2)
    z1, z2 = O.triples_residual(eps, L, t1, np.zeros_like(t2))
    assert np.abs(z1).max() == 0.0 and np.abs(z2).max() == 0.0
    s1, s2 = O.triples_residual(eps, L, t1, 1.7 * t2)
    assert rel(s1, 1.7 * o1) < 1e-13 and rel(s2, 1.7 * o2) < 1e-13
    e1, e2 = O.triples_residual(2.5 * eps, L, t1, t2)
    assert rel(e1, o1 / 2.5) < 1e-13 and rel(e2, o2 / 2.5) < 1e-13
    l1, l2 = O.triples_residual(eps, 0.5 * L, t1, t2)
    assert rel(l1, o1 / 16.0) < 1e-13 and rel(l2, o2 / 16.0) < 1e-13
    assert rel(o2, o2.transpose(1, 0, 3, 2)) < 1e-14


def test_special_cases_vanish():
    """nv = 1 or no = 1 leave only virtual-symmetric t3 (tau~ = 0), so Omega = 0."""
    for no, nv in [(4, 1), (1, 6)]:
        d = make_inputs(no, nv, 8)
        o1, o2 = O.triples_residual(d["eps"], d["L"], d["t1"], d["t2"])
        b1, b2, tau = residual_bruteforce(d["eps"], d["L"], d["t1"], d["t2"])
        assert np.abs(tau).max() > 0.0
        assert np.abs(o1).max() < 1e-18 and np.abs(o2).max() < 1e-18
        assert np.abs(b2).max() < 1e-18


def test_all_equal_triples_contribute_nothing():
    """i == j == k: tau~ is identically zero, so including those triples changes nothing."""
    d = make_inputs(4, 6, 12)
    blk, F = _blocks(d)
    for i in range(4):
        tt = O.contravariant(O.t3_amplitudes(i, i, i, d["eps"], d["t2"], blk))
        assert np.abs(tt).max() < 1e-18
    base = O.unordered_triples(4)
    with_diag = base + [(i, i, i) for i in range(4)]
    a1, a2 = O.omega_tilde(d["eps"], d["t2"], blk, F, triples=base)
    b1, b2 = O.omega_tilde(d["eps"], d["t2"], blk, F, triples=with_diag)
    assert rel(a1, b1) == 0.0 and rel(a2, b2) == 0.0


def test_triple_count_and_subset_additivity():
    """The restricted loop visits C(no+2,3) - no triples; disjoint subsets sum to the whole."""
    for no in range(1, 9):
        assert len(O.unordered_triples(no)) == comb(no + 2, 3) - no
    d = make_inputs(5, 6, 12)
    blk, F = _blocks(d)
    allt = O.unordered_triples(5)
    w1, w2 = O.omega_tilde(d["eps"], d["t2"], blk, F)
    p1, p2 = O.omega_tilde(d["eps"], d["t2"], blk, F, triples=allt[::2])
    q1, q2 = O.omega_tilde(d["eps"], d["t2"], blk, F, triples=allt[1::2])
    assert rel(p1 + q1, w1) < 1e-13 and rel(p2 + q2, w2) < 1e-13


def test_t1_transform_is_a_similarity():
    """Lt^J = (1+t)^{-1} L^J (1+t): traces and spectra are kept, the ov block is untouched,
    t1 = 0 is the identity, and the four-index transformation of g agrees."""
    d = make_inputs(3, 5, 6)
    L, t1 = d["L"], d["t1"] * 50.0
    Lt = O.t1_transform(L, t1)
    no = 3
    for J in range(L.shape[0]):
        assert abs(np.trace(Lt[J]) - np.trace(L[J])) < 1e-13
        assert abs(np.trace(Lt[J] @ Lt[J]) - np.trace(L[J] @ L[J])) < 1e-13
        ev_a = np.sort_complex(np.linalg.eigvals(Lt[J]))
        ev_b = np.sort_complex(np.linalg.eigvals(L[J]))
        assert np.abs(ev_a - ev_b).max() < 1e-10
    assert np.array_equal(Lt[:, :no, no:], L[:, :no, no:])
    assert np.array_equal(O.t1_transform(L, np.zeros_like(t1)), L)
    gt, _ = transformed_hamiltonian(d["eps"], L, t1)
    assert rel(np.einsum("Jpq,Jrs->pqrs", Lt, Lt), gt) < 1e-13


def test_fock_ov_from_full_transformation():
    """F_kc = sum_ld t^d_l (2 g_kcld - g_kdlc) is the ov block of the T1-transformed
    Fock matrix of a canonical reference (built here from h and the full g~); t1 = 0 gives 0."""
    d = make_inputs(4, 6, 10)
    t1 = d["t1"] * 30.0
    _, Ft = transformed_hamiltonian(d["eps"], d["L"], t1)
    F = O.fock_ov(d["L"], t1)
    assert np.abs(F).max() > 1e-4
    assert rel(F, Ft[:4, 4:]) < 1e-12
    assert np.abs(O.fock_ov(d["L"], np.zeros_like(t1))).max() == 0.0


def test_blocks_form_equals_cholesky_form():
    d = make_inputs(4, 6, 12)
    blk, F = _blocks(d)
    a1, a2 = O.triples_residual(d["eps"], d["L"], d["t1"], d["t2"])
    b1, b2 = O.triples_residual_blocks(d["eps"], blk.full_vvvo(), blk.g_oovo, blk.g_ovov,
                                       blk.g_ooov, blk.full_vvov(), F, d["t2"])
    assert rel(a1, b1) < 1e-15 and rel(a2, b2) < 1e-15


def oracle_flop_formula(no, nv):
    """FLOP of the oracle's contractions, written from the algorithm's shapes:
    per unordered triple, six B terms (2nv^4 + 2nv^3 no each) and, per distinct
    permutation, the four contractions 2nv^3 + 2nv^3 + 2nv^3 no + 2nv^4."""
    D, E = comb(no, 3), no * (no - 1)
    w = 6 * (2 * nv**4 + 2 * nv**3 * no)
    perm = 2 * nv**3 + 2 * nv**3 + 2 * nv**3 * no + 2 * nv**4
    return (D + E) * w + (6 * D + 3 * E) * perm


@pytest.mark.parametrize("no,nv", [(3, 4), (4, 5), (5, 3)])
def test_flop_counter(no, nv):
    d = make_inputs(no, nv, 8)
    blk, F = _blocks(d)
    fc = O.FlopCounter()
    O.omega_tilde(d["eps"], d["t2"], blk, F, flops=fc)
    assert fc.total == oracle_flop_formula(no, nv)


def test_flop_convention_reproduces_paper_efficiencies():
    """4 nv^4 no^3 FLOP per call reproduces the printed efficiencies of Tables 4 and 7
    (within the rounding of the printed minutes and percentages)."""
    with open(os.path.join(GOLDEN, "paper_timings.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        fl = O.nominal_flops(c["no"], c["nv"])
        lo = fl / ((c["minutes_per_call"] + 0.5) * 60.0) / (c["peak_gflops"] * 1e9) * 100.0
        hi = fl / ((c["minutes_per_call"] - 0.5) * 60.0) / (c["peak_gflops"] * 1e9) * 100.0
        p = c["printed_efficiency_percent"]
        assert lo - 0.05 <= p <= hi + 0.05, (c["table"], lo, hi)
    # the leading term of the algorithm's dominant contractions approaches 4 nv^4 no^3
    no, nv = 200, 10
    D, E = comb(no, 3), no * (no - 1)
    lead = (D + E) * 6 * 2 * nv**4 + (6 * D + 3 * E) * 2 * nv**4
    assert abs(lead / O.nominal_flops(no, nv) - 1.0) < 0.03


# ---------------------------------------------------------------------------
# Algorithm 2: t3-dependent intermediates of the preparation for the Jacobian
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("no,nv,nJ,t1z", [(3, 4, 6, True), (3, 4, 6, False), (4, 5, 8, False),
                                          (4, 6, 9, False), (2, 3, 5, False)])
def test_jacobian_prep_equals_bruteforce(no, nv, nJ, t1z):
    """The restricted loop of Algorithm 2 (6/3 distinct permutations, i = j = k skipped)
    against the plain definition over every ordered triple."""
    d = make_inputs(no, nv, nJ, t1_zero=t1z)
    zv, zo = O.jacobian_prep(d["eps"], d["L"], d["t1"], d["t2"])
    bv, bo = B.jacobian_prep_bruteforce(d["eps"], d["L"], d["t1"], d["t2"])
    assert np.abs(bv).max() > 0 and np.abs(bo).max() > 0
    assert np.abs(zv - bv).max() <= 1e-13 * np.abs(bv).max()
    assert np.abs(zo - bo).max() <= 1e-13 * np.abs(bo).max()


def test_jacobian_prep_trace_is_omega1():
    """sum_j Z~^o_{ajij} = sum_{jkbc} tau~^{abc}_{ijk} g_{jbkc}, the Omega1 contraction of
    Algorithm 1 (computed here by the other routine)."""
    d = make_inputs(5, 9, 14)
    zv, zo = O.jacobian_prep(d["eps"], d["L"], d["t1"], d["t2"])
    o1, _ = O.omega_tilde_subset(d["eps"], d["L"], d["t1"], d["t2"], O.unordered_triples(5))
    tr = np.einsum("ajij->ia", zo)
    assert np.abs(tr - o1).max() <= 1e-13 * np.abs(o1).max()


def test_jacobian_prep_homogeneity_and_special_cases():
    """Linear in t2; L -> s L scales both intermediates by s^4; t2 = 0 and no = 1 give 0."""
    d = make_inputs(4, 6, 9)
    zv, zo = O.jacobian_prep(d["eps"], d["L"], d["t1"], d["t2"])
    zv2, zo2 = O.jacobian_prep(d["eps"], d["L"], d["t1"], 2.0 * d["t2"])
    assert np.abs(zv2 - 2.0 * zv).max() <= 1e-14 * np.abs(zv).max()
    assert np.abs(zo2 - 2.0 * zo).max() <= 1e-14 * np.abs(zo).max()
    zv3, zo3 = O.jacobian_prep(d["eps"], 1.5 * d["L"], d["t1"], d["t2"])
    assert np.abs(zv3 - 1.5 ** 4 * zv).max() <= 1e-13 * np.abs(zv3).max()
    assert np.abs(zo3 - 1.5 ** 4 * zo).max() <= 1e-13 * np.abs(zo3).max()
    zv0, zo0 = O.jacobian_prep(d["eps"], d["L"], d["t1"], 0.0 * d["t2"])
    assert not zv0.any() and not zo0.any()
    e = make_inputs(1, 5, 7)
    zv1, zo1 = O.jacobian_prep(e["eps"], e["L"], e["t1"], e["t2"])
    assert not zv1.any() and not zo1.any()


# --------------------------------------------------------------------------
# Algorithm 3: the triples contributions to the transition densities.
# --------------------------------------------------------------------------

def _alg3(no, nv, nJ, t1z=False, scale_l=1.0, zero_l1=False, zero_l2=False, zero_t2=False):
    from paper_2007_01088_amd.synth import make_left_inputs
    d = make_inputs(no, nv, nJ, t1_zero=t1z)
    lf = make_left_inputs(no, nv)
    l1 = 0.0 * lf["l1"] if zero_l1 else scale_l * lf["l1"]
    l2 = 0.0 * lf["l2"] if zero_l2 else scale_l * lf["l2"]
    t2 = 0.0 * d["t2"] if zero_t2 else d["t2"]
    return d, l1, l2, t2, lf["omega"]


@pytest.mark.parametrize("no,nv,nJ,t1z", [(3, 4, 6, False), (4, 5, 8, False), (4, 3, 5, True),
                                          (2, 6, 9, False), (5, 3, 7, False)])
def test_transition_density_loops_equal_bruteforce(no, nv, nJ, t1z):
    """Algorithm 3's two restricted loops (occupied i >= j >= k for D_cd, D_kc, Y^o, D_ld;
    virtual a >= b >= c for D_lk, with t3 and L3 built for fixed virtual indices) reach the
    plain definition over all ordered index tuples with full T3 and L3 tensors, whose
    integrals come from the full four-index T1 transformation."""
    d, l1, l2, t2, w = _alg3(no, nv, nJ, t1z)
    got = O.transition_density(d["eps"], d["L"], d["t1"], t2, l1, l2, w)
    Lt = O.t1_transform(d["L"], d["t1"])
    blk = O.IntegralBlocks(Lt, no)
    F = O.fock_ov(d["L"], d["t1"])
    Y = O.transition_density_occupied(d["eps"], t2, l1, l2, w, blk, F)[3]
    ref = B.transition_density_bruteforce(d["eps"], d["L"], d["t1"], t2, l1, l2, w)
    for name, g, r in zip(("D_cd", "D_kc", "D_ld", "D_lk", "Y^o"), list(got) + [Y], ref):
        assert np.abs(r).max() > 0, name
        assert rel(g, r) < 1e-12, (name, rel(g, r))


@pytest.mark.parametrize("no,nv,nJ", [(4, 6, 10), (6, 4, 8), (3, 9, 12)])
def test_transition_density_trace_identity(no, nv, nJ):
    """tr D_vv = (1/2) sum L~ t3 = - tr D_oo: the occupied loop's D_cd and the virtual loop's
    D_lk (separate t3 and L3 builders) must cancel in the trace."""
    d, l1, l2, t2, w = _alg3(no, nv, nJ)
    D_cd, _, _, D_lk = O.transition_density(d["eps"], d["L"], d["t1"], t2, l1, l2, w)
    tv, to = np.trace(D_cd), np.trace(D_lk)
    assert abs(tv) > 0
    assert abs(tv + to) <= 1e-12 * abs(tv), (tv, to)


def test_l3_permutational_symmetry():
    """L^{abc}_{ijk} = L^{bac}_{jik} = L^{cba}_{kji} = L^{acb}_{ikj} = L^{cab}_{kij} = L^{bca}_{jki}
    (P^{abc}_{ijk} symmetrises the builder), checked on an all-distinct triple."""
    from paper_2007_01088_amd.synth import make_left_inputs
    d = make_inputs(4, 5, 8)
    lf = make_left_inputs(4, 5)
    blk, F = _blocks(d)
    args = (lf["omega"], d["eps"], lf["l1"], lf["l2"], blk, F)
    ref = O.l3_amplitudes(3, 1, 0, *args)
    for (i, j, k), lab in (((1, 3, 0), "bac"), ((0, 1, 3), "cba"), ((3, 0, 1), "acb"),
                           ((0, 3, 1), "cab"), ((1, 0, 3), "bca")):
        other = O.l3_amplitudes(i, j, k, *args)
        assert rel(np.einsum(lab + "->abc", other), ref) < 1e-13, (i, j, k)


def test_transition_density_linearity_and_special_cases():
    """The densities are linear in the left amplitudes (L3 is), vanish without them or
    without t2 (t3 = 0), and vanish for a single occupied or virtual orbital (every
    contravariant L3 with all-equal indices is zero)."""
    no, nv, nJ = 3, 4, 6
    d, l1, l2, t2, w = _alg3(no, nv, nJ)
    full = O.transition_density(d["eps"], d["L"], d["t1"], t2, l1, l2, w)
    only1 = O.transition_density(d["eps"], d["L"], d["t1"], t2, l1, 0.0 * l2, w)
    only2 = O.transition_density(d["eps"], d["L"], d["t1"], t2, 0.0 * l1, l2, w)
    twice = O.transition_density(d["eps"], d["L"], d["t1"], t2, 2.0 * l1, 2.0 * l2, w)
    for f, a, b, t in zip(full, only1, only2, twice):
        assert rel(a + b, f) < 1e-12
        assert rel(t, 2.0 * f) < 1e-12
    for x in O.transition_density(d["eps"], d["L"], d["t1"], 0.0 * t2, l1, l2, w):
        assert not np.any(x)
    for x in O.transition_density(d["eps"], d["L"], d["t1"], t2, 0.0 * l1, 0.0 * l2, w):
        assert not np.any(x)
    for (n_o, n_v) in ((1, 4), (3, 1)):
        d1, a1, a2, b2, w1 = _alg3(n_o, n_v, 5)
        for x in O.transition_density(d1["eps"], d1["L"], d1["t1"], b2, a1, a2, w1):
            assert np.abs(x).max() < 1e-18
