"""Plain FP64 CPU oracle for the CC3 ground-state triples residual.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the HIP
library and its Python binding) never calls it and shares no code with it.

It follows Paul, Myhre & Koch, "A new and efficient implementation of CC3"
(arXiv 2007.01088): Section "Implementation", Algorithm 1 (CC3 ground-state
equations), the permutation operator P^{abc}_{ijk}, the orbital-energy
difference, the contravariant amplitudes and the covariant back-transformation;
Algorithm 2 (the t3-dependent intermediates of the preparation for the
Jacobian transformations); and Algorithm 3 (the triples contributions to the
transition densities D^{m,0}: the occupied loop for the vv, ov and vo blocks and
the loop over the virtual indices for the oo block).
Every step is a numpy einsum over float64 arrays, with no blocking or fusion.
The residual is written as its definition, a sum over every ordered occupied
triple (p, q, r) of contributions of the contravariant amplitudes of that
triple; the ordered triples are visited grouped by their sorted form, whose
amplitudes are built once (the restricted loop i >= j >= k) and relabelled for
the other orderings by the permutational symmetry of t3.

Readings of the paper used here (each is listed in the design notes):
  * The T1 transformation (Sec. Theory, H = exp(-T1) H exp(T1)) acts on the
    Cholesky vectors as  Lt^J = (1 - t) L^J (1 + t)  with t[no+a][i] = t^a_i.
  * F_kc is the ov block of the T1-transformed Fock matrix of a canonical
    Hartree-Fock reference (whose own ov block vanishes):
        F_kc = sum_{ld} t^d_l (2 g_kcld - g_kdlc)   (untransformed ov integrals).
  * The contravariant amplitudes permute the virtual indices only, at fixed
    (i,j,k), as in the second statement of Algorithm 1.  (The displayed
    equation that permutes occupied and virtual indices together would be
    identically zero under the permutational symmetry.)
  * The denominator uses the canonical orbital energies:
        eps^{abc}_{ijk} = e_a + e_b + e_c - e_i - e_j - e_k,  tau = -X / eps.
  * For two equal occupied indices each distinct occupied permutation is
    applied once (three of them); i == j == k is skipped (tau-tilde vanishes).
  * Back-transformation  Omega^{ab}_{ij} = 1/3 P^{ab}_{ij}(2 Ot^{ab}_{ij} + Ot^{ba}_{ij})
    with P^{ab}_{ij} Y^{ab}_{ij} = Y^{ab}_{ij} + Y^{ba}_{ji}, on full square
    storage.  Absolute agreement with the paper's program at the diagonal
    (ai == bj) elements is parity unpinned: the paper prints no residual values.

Array layouts (row-major): eps[no+nv] (occupied first), L[nJ][nmo][nmo],
t1[no][nv] = t^a_i, t2[no][no][nv][nv] = t^{ab}_{ij}, omega1[no][nv],
omega2[no][no][nv][nv]; integral blocks in the paper's index order,
g_vvvo[b][d][c][k] = g_{bdck}, g_oovo[l][j][c][k] = g_{ljck},
g_ovov[j][b][k][c] = g_{jbkc}, g_ooov[j][l][k][c] = g_{jlkc},
g_vvov[d][b][k][c] = g_{dbkc}, F[k][c].
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "t1_transform", "IntegralBlocks", "fock_ov", "w_term", "t3_amplitudes",
    "contravariant", "orderings", "relabel", "occupied_permutations", "unordered_triples",
    "omega_tilde",
    "back_transform", "triples_residual", "triples_residual_blocks",
    "omega_tilde_subset", "nominal_flops", "FlopCounter", "jacobian_prep_tilde",
    "jacobian_prep", "l3_amplitudes", "virtual_triples", "transition_density_occupied",
    "transition_density_virtual", "transition_density",
]


class FlopCounter:
    """Counts 2*M*N*K for every contraction the oracle executes."""

    def __init__(self) -> None:
        self.total = 0

    def add(self, n: int) -> None:
        self.total += int(n)


def _e(spec: str, *ops, flops: FlopCounter | None = None):
    """einsum with the FLOP count of a plain contraction: 2 * (output size) * (summed size)."""
    if flops is not None:
        ins, out = spec.split("->")
        dims = {}
        for lab, op in zip(ins.split(","), ops):
            for ch, n in zip(lab, op.shape):
                dims[ch] = n
        summed = [ch for ch in dims if ch not in out]
        osz = int(np.prod([dims[ch] for ch in out])) if out else 1
        ssz = int(np.prod([dims[ch] for ch in summed])) if summed else 1
        if summed:
            flops.add(2 * osz * ssz)
    return np.einsum(spec, *ops, optimize=True)


# --------------------------------------------------------------------------
# Integrals in the T1-transformed basis (Sec. Theory, eq. for H = e^{-T1} H e^{T1};
# Sec. Implementation: "integrals in T1-transformed basis").
# --------------------------------------------------------------------------

def t1_transform(L: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """Lt^J = (1 - t) L^J (1 + t) with t[no+a][i] = t^a_i (all other entries zero).

    exp(-T1) a_p^dagger exp(T1) = sum_q a_q^dagger (1 - t)_{qp} and
    exp(-T1) a_q exp(T1) = sum_s a_s (1 + t)_{qs}^T, so every one-index object
    h_pq becomes ((1 - t) h (1 + t))_pq; the Cholesky factors transform alike.
    """
    nJ, nmo, _ = L.shape
    no, nv = t1.shape
    t = np.zeros((nmo, nmo))
    t[no:, :no] = t1.T
    left = np.eye(nmo) - t
    right = np.eye(nmo) + t
    return np.ascontiguousarray(np.matmul(np.matmul(left, L), right))


class IntegralBlocks:
    """Integral blocks g_pqrs = sum_J Lt^J_pq Lt^J_rs needed by Algorithm 1.

    The two nv^3 no blocks (vv|vo) and (vv|ov) are built one occupied slab at a
    time on demand (g_vvvo[:, :, :, k] and g_vvov[:, :, k, :]), so a sampled
    subset of triples needs only the slabs of its occupied indices.
    """

    def __init__(self, Lt: np.ndarray, no: int, full: bool = False):
        self.no = no
        self.nv = Lt.shape[1] - no
        o, v = slice(0, no), slice(no, None)
        self.L_vv = Lt[:, v, v]
        self.L_vo = Lt[:, v, o]
        self.L_oo = Lt[:, o, o]
        self.L_ov = Lt[:, o, v]
        # the small blocks, complete
        self.g_oovo = _e("Jlj,Jck->ljck", self.L_oo, self.L_vo)
        self.g_ovov = _e("Jjb,Jkc->jbkc", self.L_ov, self.L_ov)
        self.g_ooov = _e("Jjl,Jkc->jlkc", self.L_oo, self.L_ov)
        self._vvvo: dict[int, np.ndarray] = {}
        self._vvov: dict[int, np.ndarray] = {}
        if full:
            for k in range(no):
                self.vvvo(k)
                self.vvov(k)

    def vvvo(self, k: int) -> np.ndarray:
        """g_vvvo[b][d][c] at fixed k: g_{bdck}."""
        if k not in self._vvvo:
            self._vvvo[k] = _e("Jbd,Jc->bdc", self.L_vv, self.L_vo[:, :, k])
        return self._vvvo[k]

    def vvov(self, k: int) -> np.ndarray:
        """g_vvov[d][b][c] at fixed k: g_{dbkc}."""
        if k not in self._vvov:
            self._vvov[k] = _e("Jdb,Jc->dbc", self.L_vv, self.L_ov[:, k, :])
        return self._vvov[k]

    @classmethod
    def from_arrays(cls, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov):
        """Blocks given directly in the paper's index order (the integral-blocks form)."""
        self = cls.__new__(cls)
        self.no = g_oovo.shape[0]
        self.nv = g_vvvo.shape[0]
        self.g_oovo, self.g_ovov, self.g_ooov = g_oovo, g_ovov, g_ooov
        self._vvvo = {k: np.ascontiguousarray(g_vvvo[:, :, :, k]) for k in range(self.no)}
        self._vvov = {k: np.ascontiguousarray(g_vvov[:, :, k, :]) for k in range(self.no)}
        return self

    def ovvv(self, i: int) -> np.ndarray:
        """g_ovvv[b][d][c] at fixed i: g_{ibdc} (Algorithm 3's L3 builder)."""
        return _e("Jb,Jdc->bdc", self.L_ov[:, i, :], self.L_vv)

    def full_vvvo(self) -> np.ndarray:
        return np.stack([self.vvvo(k) for k in range(self.no)], axis=3)

    def full_vvov(self) -> np.ndarray:
        return np.stack([self.vvov(k) for k in range(self.no)], axis=2)


def fock_ov(L: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """F_kc of the T1-transformed Fock matrix (canonical HF reference, whose ov block is zero).

    F_kc = h~_kc + sum_l (2 g~_kcll - g~_kllc); with the ov block of Lt equal to
    the untransformed one this reduces to sum_{ld} t^d_l (2 g_kcld - g_kdlc).
    """
    no, nv = t1.shape
    Lov = L[:, :no, no:]
    g_ovov = _e("Jkc,Jld->kcld", Lov, Lov)
    return np.ascontiguousarray(2.0 * _e("ld,kcld->kc", t1, g_ovov) - _e("ld,kdlc->kc", t1, g_ovov))


# --------------------------------------------------------------------------
# Algorithm 1, inside the restricted loop over i >= j >= k.
# --------------------------------------------------------------------------

def w_term(p: int, q: int, r: int, t2: np.ndarray, blk: IntegralBlocks,
           flops: FlopCounter | None = None) -> np.ndarray:
    """B^{abc}_{pqr} = sum_d t^{ad}_{pq} g_{bdcr} - sum_l t^{ab}_{pl} g_{lqcr}   (Algorithm 1, first statement)."""
    vv = _e("ad,bdc->abc", t2[p, q], blk.vvvo(r), flops=flops)
    oo = _e("lab,lc->abc", t2[p], blk.g_oovo[:, q, :, r], flops=flops)
    return vv - oo


def t3_amplitudes(i: int, j: int, k: int, eps: np.ndarray, t2: np.ndarray,
                  blk: IntegralBlocks, flops: FlopCounter | None = None) -> np.ndarray:
    """tau^{abc}_{ijk} = -(eps^{abc}_{ijk})^{-1} P^{abc}_{ijk} B^{abc}_{ijk}.

    P^{abc}_{ijk} B = B^{abc}_{ijk} + B^{bac}_{jik} + B^{cba}_{kji} + B^{acb}_{ikj}
                    + B^{bca}_{jki} + B^{cab}_{kij}   (the permutation operator of Sec. Implementation).
    """
    no = t2.shape[0]
    X = (w_term(i, j, k, t2, blk, flops)
         + np.einsum("bac->abc", w_term(j, i, k, t2, blk, flops))
         + np.einsum("cba->abc", w_term(k, j, i, t2, blk, flops))
         + np.einsum("acb->abc", w_term(i, k, j, t2, blk, flops))
         + np.einsum("bca->abc", w_term(j, k, i, t2, blk, flops))
         + np.einsum("cab->abc", w_term(k, i, j, t2, blk, flops)))
    ev = eps[no:]
    D = (ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
         - eps[i] - eps[j] - eps[k])
    return -X / D


def contravariant(tau: np.ndarray) -> np.ndarray:
    """tau~^{abc} = 4 tau^{abc} - 2 tau^{acb} - 2 tau^{cba} - 2 tau^{bac} + tau^{bca} + tau^{cab} (fixed ijk)."""
    return (4.0 * tau
            - 2.0 * np.einsum("acb->abc", tau)
            - 2.0 * np.einsum("cba->abc", tau)
            - 2.0 * np.einsum("bac->abc", tau)
            + np.einsum("bca->abc", tau)
            + np.einsum("cab->abc", tau))


def orderings(i: int, j: int, k: int):
    """The distinct ordered triples (p, q, r) made of the occupied indices i, j, k, each with
    the axis permutation perm that gives it: (p, q, r) = ((i, j, k)[perm[0]], ...).  Six when
    i, j, k differ, three when two are equal, one when all three are."""
    base = (i, j, k)
    out, seen = [], set()
    for perm in itertools.permutations(range(3)):
        pqr = tuple(base[m] for m in perm)
        if pqr not in seen:
            seen.add(pqr)
            out.append((pqr, perm))
    return out


def relabel(block: np.ndarray, perm) -> np.ndarray:
    """X_{pqr} from X_{ijk} for (p,q,r) = (i,j,k) taken in the order perm.

    By the permutational symmetry of Sec. Implementation, tau^{abc}_{ijk} is unchanged
    when the pairs (a,i), (b,j), (c,k) are permuted together; so the virtual index paired
    with the m-th occupied index of (p,q,r) sits on axis perm[m] of X_{ijk}:
    X_{pqr}[a0, a1, a2] = X_{ijk}[y] with y[perm[m]] = a_m, which is numpy's transpose.
    The contravariant amplitudes share the symmetry (their coefficients are the same for
    every relabelling), and so do the left-state amplitudes of Algorithm 3."""
    return np.transpose(block, perm)


def occupied_permutations(i: int, j: int, k: int, tt: np.ndarray):
    """[((p,q,r), X_{pqr})] over the distinct orderings of (i,j,k), X_{ijk} = tt."""
    return [(pqr, relabel(tt, perm)) for pqr, perm in orderings(i, j, k)]


def unordered_triples(no: int):
    """The restricted loop i >= j >= k of Algorithm 1, without the i == j == k triples."""
    return [(i, j, k) for i in range(no) for j in range(i + 1) for k in range(j + 1)
            if not (i == j == k)]


def omega_tilde(eps: np.ndarray, t2: np.ndarray, blk: IntegralBlocks, F: np.ndarray,
                triples=None, flops: FlopCounter | None = None):
    """The contravariant residual of the CC3 ground-state equations (Algorithm 1).

    By definition it sums, over every ordered occupied triple (p, q, r) (those with
    p == q == r contribute nothing: their contravariant amplitudes vanish), with
    U = tau~_{pqr}:
        Ot1[p][a]    = sum_{bc} U[a,b,c] g_{qbrc}
        Ot2[p][q][a][b] = sum_c U[a,b,c] F_{rc}
        Ot2[p][l][a][b] = - sum_c U[a,b,c] g_{qlrc}       for every l
        Ot2[p][q][a][d] = sum_{bc} U[a,b,c] g_{dbrc}      for every d
    (each line adds into the named block).  `triples` lists unordered triples
    i >= j >= k (default: all of them); each stands for its distinct orderings, whose
    amplitudes are the relabelled amplitudes of the sorted triple.
    """
    no, _, nv, _ = t2.shape
    Ot1 = np.zeros((no, nv))
    Ot2 = np.zeros((no, no, nv, nv))
    if triples is None:
        triples = unordered_triples(no)
    for rep in triples:
        i, j, k = (int(x) for x in rep)
        if i == j == k:
            continue
        tt = contravariant(t3_amplitudes(i, j, k, eps, t2, blk, flops))
        for (p, q, r), perm in orderings(i, j, k):
            U = relabel(tt, perm)
            Ot1[p] += _e("abc,bc->a", U, blk.g_ovov[q, :, r, :], flops=flops)
            Ot2[p, q] += _e("abc,c->ab", U, F[r], flops=flops)
            Ot2[p] -= _e("abc,lc->lab", U, blk.g_ooov[q, :, r, :], flops=flops)
            Ot2[p, q] += _e("abc,dbc->ad", U, blk.vvov(r), flops=flops)
    return Ot1, Ot2


def back_transform(Ot1: np.ndarray, Ot2: np.ndarray):
    """Omega^a_i = Ot^a_i;  Omega^{ab}_{ij} = 1/3 P^{ab}_{ij} (2 Ot^{ab}_{ij} + Ot^{ba}_{ij})."""
    Y = 2.0 * Ot2 + np.einsum("ijba->ijab", Ot2)
    return Ot1.copy(), (Y + np.einsum("jiba->ijab", Y)) / 3.0


# --------------------------------------------------------------------------
# Whole calls.
# --------------------------------------------------------------------------

def triples_residual(eps, L, t1, t2, flops: FlopCounter | None = None):
    """One evaluation of the CC3 triples contribution (Omega1, Omega2) from Cholesky vectors."""
    no = t1.shape[0]
    Lt = t1_transform(L, t1)
    blk = IntegralBlocks(Lt, no)
    F = fock_ov(L, t1)
    return back_transform(*omega_tilde(eps, t2, blk, F, flops=flops))


def triples_residual_blocks(eps, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F, t2):
    """The same evaluation from integral blocks given in the paper's index order."""
    blk = IntegralBlocks.from_arrays(g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov)
    return back_transform(*omega_tilde(eps, t2, blk, F))


def omega_tilde_subset(eps, L, t1, t2, triples):
    """Contravariant (Ot1, Ot2) from a listed subset of unordered triples only (no back-transform)."""
    no = t1.shape[0]
    Lt = t1_transform(L, t1)
    blk = IntegralBlocks(Lt, no)
    F = fock_ov(L, t1)
    return omega_tilde(eps, t2, blk, F, triples=[tuple(t) for t in triples])


def nominal_flops(no: int, nv: int) -> float:
    """The paper's asymptotic ground-state cost per residual call: 4 nv^4 no^3 FLOP (abstract)."""
    return 4.0 * float(nv) ** 4 * float(no) ** 3


# --------------------------------------------------------------------------
# Preparation for the Jacobian transformations (Algorithm 2).
# --------------------------------------------------------------------------

def jacobian_prep_tilde(eps: np.ndarray, t2: np.ndarray, blk: IntegralBlocks, triples=None,
                        flops: FlopCounter | None = None):
    """The t3-dependent intermediates of the preparation for the Jacobian transformations
    (Algorithm 2).

    By definition they sum, over every ordered occupied triple (p, q, r), with
    U = tau~_{pqr} (the amplitudes and their contravariant form of Algorithm 1):
        Zv[a][b][p][d] -= sum_c    U[a,b,c] g_{qdrc}
        Zo[a][q][p][l] += sum_{bc} U[a,b,c] g_{lbrc}
    Arrays (row-major): Zv[a][b][i][d] = Z~^v_{abid}, Zo[a][j][i][l] = Z~^o_{ajil}.
    `triples` lists unordered triples, each standing for its distinct orderings.
    """
    no, _, nv, _ = t2.shape
    Zv = np.zeros((nv, nv, no, nv))
    Zo = np.zeros((nv, no, no, no))
    if triples is None:
        triples = unordered_triples(no)
    for rep in triples:
        i, j, k = (int(x) for x in rep)
        if i == j == k:
            continue
        tt = contravariant(t3_amplitudes(i, j, k, eps, t2, blk, flops))
        for (p, q, r), perm in orderings(i, j, k):
            U = relabel(tt, perm)
            Zv[:, :, p, :] -= _e("abc,dc->abd", U, blk.g_ovov[q, :, r, :], flops=flops)
            Zo[:, q, p, :] += _e("abc,lbc->al", U, blk.g_ovov[:, :, r, :], flops=flops)
    return Zv, Zo


def jacobian_prep(eps, L, t1, t2, flops: FlopCounter | None = None):
    """Algorithm 2 from Cholesky vectors: (Zv, Zo) as in jacobian_prep_tilde, all triples."""
    no = t1.shape[0]
    Lt = t1_transform(L, t1)
    blk = IntegralBlocks(Lt, no)
    return jacobian_prep_tilde(eps, t2, blk, flops=flops)


# --------------------------------------------------------------------------
# Contributions of the triples to the transition densities (Algorithm 3).
#
# Readings (each is listed in the design notes): the amplitudes written with t
# and with tau in the algorithm are the same ground-state amplitudes (t3 by the
# first statement of Algorithm 1, t2 the doubles); L^a_i, L^{ab}_{ij} are the
# left-state singles and doubles, L^{ab}_{ij} = L^{ba}_{ji}; omega is the
# excitation energy; the integrals and F are the T1-transformed ones of
# Algorithm 1; "for permutations" applies each distinct permutation once, and
# the all-equal triples (i == j == k, a == b == c) are skipped, their
# contravariant amplitudes vanishing.  Array layouts: D_cd[c][d], D_kc[k][c],
# D_ld[l][d], D_lk[l][k], Y^o[c][l][i][k].
# --------------------------------------------------------------------------

def l3_term(p: int, q: int, r: int, l1: np.ndarray, l2: np.ndarray, blk: IntegralBlocks,
            F: np.ndarray) -> np.ndarray:
    """C^{abc}_{pqr} = L^a_p g_{qbrc} + L^{ab}_{pq} F_{rc} + sum_d L^{ad}_{qr} g_{pbdc}
    - sum_l L^{ab}_{lr} g_{plqc}   (Algorithm 3, second statement, before P)."""
    return (_e("a,bc->abc", l1[p], blk.g_ovov[q, :, r, :])
            + _e("ab,c->abc", l2[p, q], F[r])
            + _e("ad,bdc->abc", l2[q, r], blk.ovvv(p))
            - _e("lab,lc->abc", l2[:, r], blk.g_ooov[p, :, q, :]))


def l3_amplitudes(i: int, j: int, k: int, omega: float, eps: np.ndarray, l1: np.ndarray,
                  l2: np.ndarray, blk: IntegralBlocks, F: np.ndarray) -> np.ndarray:
    """L^{abc}_{ijk} = (omega - eps^{abc}_{ijk})^{-1} P^{abc}_{ijk} C^{abc}_{ijk}, with the
    permutation operator of Algorithm 1."""
    no = l1.shape[0]
    X = (l3_term(i, j, k, l1, l2, blk, F)
         + np.einsum("bac->abc", l3_term(j, i, k, l1, l2, blk, F))
         + np.einsum("cba->abc", l3_term(k, j, i, l1, l2, blk, F))
         + np.einsum("acb->abc", l3_term(i, k, j, l1, l2, blk, F))
         + np.einsum("bca->abc", l3_term(j, k, i, l1, l2, blk, F))
         + np.einsum("cab->abc", l3_term(k, i, j, l1, l2, blk, F)))
    ev = eps[no:]
    D = (ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
         - eps[i] - eps[j] - eps[k])
    return X / (omega - D)


def transition_density_occupied(eps, t2, l1, l2, omega, blk: IntegralBlocks, F, triples=None):
    """The occupied-index loop of Algorithm 3: D_cd, D_kc, then D_ld from Y^o.

    With tau_{pqr} the ground-state amplitudes (Algorithm 1), L_{pqr} the left-state
    triples (l3_amplitudes), and L~, tau~ their contravariant forms, the contributions
    sum over every ordered occupied triple (p, q, r):
        Y^o[c][l][p][r] += sum_{ab} L~_{pqr}[a,b,c] t2[l][q][a][b]
        D_cd[c][d]      += 1/2 sum_{ab} L~_{pqr}[a,b,c] tau_{pqr}[a,b,d]
        D_kc[r][c]      += sum_{ab} l2[p][q][a][b] tau~_{pqr}[a,b,c]
    and after the sum  D_ld[l][d] = - sum_{cik} Y^o[c][l][i][k] t2[k][i][c][d].
    `triples` lists unordered triples, each standing for its distinct orderings.
    Returns (D_cd, D_kc, D_ld, Y^o)."""
    no, _, nv, _ = t2.shape
    D_cd = np.zeros((nv, nv))
    D_kc = np.zeros((no, nv))
    Y = np.zeros((nv, no, no, no))
    if triples is None:
        triples = unordered_triples(no)
    for rep in triples:
        i, j, k = (int(x) for x in rep)
        if i == j == k:
            continue
        tau = t3_amplitudes(i, j, k, eps, t2, blk)
        tt = contravariant(tau)
        lt = contravariant(l3_amplitudes(i, j, k, omega, eps, l1, l2, blk, F))
        for (p, q, r), perm in orderings(i, j, k):
            LT, T, TT = relabel(lt, perm), relabel(tau, perm), relabel(tt, perm)
            Y[:, :, p, r] += _e("abc,lab->cl", LT, t2[:, q])
            D_cd += 0.5 * _e("abc,abd->cd", LT, T)
            D_kc[r] += _e("ab,abc->c", l2[p, q], TT)
    D_ld = -_e("clik,kicd->ld", Y, t2)
    return D_cd, D_kc, D_ld, Y


def virtual_triples(nv: int):
    """The loop a >= b >= c of Algorithm 3, without the a == b == c triples."""
    return [(a, b, c) for a in range(nv) for b in range(a + 1) for c in range(b + 1)
            if not (a == b == c)]


# occupied relabelling [i][j][k] that gives a block of the virtual labels (x,y,z) from
# the block of (a,b,c), by the simultaneous permutational symmetry
# X^{xyz}_{ijk} = X^{abc}_{sigma(ijk)}:  label order -> einsum source subscripts
_VPERM = (("abc", "ijk"), ("bac", "jik"), ("cba", "kji"),
          ("acb", "ikj"), ("bca", "kij"), ("cab", "jki"))


def _virtual_perm(block: np.ndarray, src: str) -> np.ndarray:
    return np.einsum(src + "->ijk", block)


def _w_virtual(x: int, y: int, z: int, t2, Gw, blk: IntegralBlocks) -> np.ndarray:
    """B^{xyz}_{ijk} over all (i,j,k): sum_d t^{xd}_{ij} g_{ydzk} - sum_l t^{xy}_{il} g_{ljzk}."""
    return (_e("ijd,dk->ijk", t2[:, :, x, :], Gw[y, :, z, :])
            - _e("il,ljk->ijk", t2[:, :, x, y], blk.g_oovo[:, :, z, :]))


def _c_virtual(x: int, y: int, z: int, l1, l2, F, Go, blk: IntegralBlocks) -> np.ndarray:
    """C^{xyz}_{ijk} over all (i,j,k): L^x_i g_{jykz} + L^{xy}_{ij} F_{kz}
    + sum_d L^{xd}_{jk} g_{iydz} - sum_l L^{xy}_{lk} g_{iljz}."""
    return (_e("i,jk->ijk", l1[:, x], blk.g_ovov[:, y, :, z])
            + _e("ij,k->ijk", l2[:, :, x, y], F[:, z])
            + _e("jkd,id->ijk", l2[:, :, x, :], Go[:, y, :, z])
            - _e("lk,ilj->ijk", l2[:, :, x, y], blk.g_ooov[:, :, :, z]))


def _p_virtual(build) -> np.ndarray:
    """P^{abc}_{ijk} for a fixed virtual triple: B^{abc}_{ijk} + B^{bac}_{jik} + B^{cba}_{kji}
    + B^{acb}_{ikj} + B^{bca}_{jki} + B^{cab}_{kij}, with build(x, y, z) giving B^{xyz} over ijk."""
    return (build(0, 1, 2) + np.einsum("jik->ijk", build(1, 0, 2))
            + np.einsum("kji->ijk", build(2, 1, 0)) + np.einsum("ikj->ijk", build(0, 2, 1))
            + np.einsum("jki->ijk", build(1, 2, 0)) + np.einsum("kij->ijk", build(2, 0, 1)))


def transition_density_virtual(eps, t2, l1, l2, omega, blk: IntegralBlocks, F, triples=None):
    """The loop over a >= b >= c of Algorithm 3: t3 and L3 for the fixed virtual triple and
    every (i,j,k), L~ by the virtual permutations at fixed (i,j,k) (as occupied
    relabellings of the block), and for each distinct permutation (x,y,z) of (a,b,c)
        D_lk -= 1/2 sum_{ij} L~^{xyz}_{ijk} t^{xyz}_{ijl}.
    Returns D_lk."""
    no, _, nv, _ = t2.shape
    Gw = blk.full_vvvo()                                              # g_{bdck}[b][d][c][k]
    Go = np.stack([blk.ovvv(i) for i in range(no)], axis=0)           # g_{ibdc}[i][b][d][c]
    eo = eps[:no]
    Dijk = eo[:, None, None] + eo[None, :, None] + eo[None, None, :]
    D_lk = np.zeros((no, no))
    if triples is None:
        triples = virtual_triples(nv)
    for (a, b, c) in triples:
        lab = (int(a), int(b), int(c))
        if lab[0] == lab[1] == lab[2]:
            continue
        ev = eps[no + lab[0]] + eps[no + lab[1]] + eps[no + lab[2]]
        tau = -_p_virtual(lambda x, y, z: _w_virtual(lab[x], lab[y], lab[z], t2, Gw, blk)) \
            / (ev - Dijk)
        lam = _p_virtual(lambda x, y, z: _c_virtual(lab[x], lab[y], lab[z], l1, l2, F, Go, blk)) \
            / (omega - (ev - Dijk))
        # L~^{abc}_{ijk} = 4 L^{abc} - 2 L^{acb} - 2 L^{cba} - 2 L^{bac} + L^{bca} + L^{cab}
        lt = (4.0 * lam - 2.0 * np.einsum("ikj->ijk", lam) - 2.0 * np.einsum("kji->ijk", lam)
              - 2.0 * np.einsum("jik->ijk", lam) + np.einsum("kij->ijk", lam)
              + np.einsum("jki->ijk", lam))
        seen = set()
        for order, src in _VPERM:
            xyz = tuple(lab["abc".index(ch)] for ch in order)
            if xyz in seen:
                continue
            seen.add(xyz)
            D_lk -= 0.5 * _e("ijk,ijl->lk", _virtual_perm(lt, src), _virtual_perm(tau, src))
    return D_lk


def transition_density(eps, L, t1, t2, l1, l2, omega):
    """Algorithm 3 from Cholesky vectors: the triples contributions (D_cd, D_kc, D_ld, D_lk)
    to D^{m,0} for the left state (l1, l2, omega)."""
    no = t1.shape[0]
    Lt = t1_transform(L, t1)
    blk = IntegralBlocks(Lt, no)
    F = fock_ov(L, t1)
    D_cd, D_kc, D_ld, _ = transition_density_occupied(eps, t2, l1, l2, omega, blk, F)
    D_lk = transition_density_virtual(eps, t2, l1, l2, omega, blk, F)
    return D_cd, D_kc, D_ld, D_lk
