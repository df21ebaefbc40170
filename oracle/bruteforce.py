"""Brute-force evaluation of the CC3 triples residual (and of the t3-dependent
intermediates of the Jacobian preparation, and of the triples contributions to the
transition densities) over the full T3 (and L3) tensors.

TEST INFRASTRUCTURE ONLY (tiny sizes: it stores all nv^3 no^3 amplitudes).
This is the plain definition the restricted loop of Algorithm 1 reaches up to
rounding order: every ordered occupied triple (i, j, k), no permutational
shortcut, and the Fock ov block obtained from a full four-index T1
transformation of a one-electron operator h chosen so that the canonical
Hartree-Fock Fock matrix is diag(eps).  It shares no code with the loop oracle
in cc3_oracle.py, against which it is compared.
"""
from __future__ import annotations

import numpy as np


def _t1_matrices(t1: np.ndarray, nmo: int):
    no, nv = t1.shape
    t = np.zeros((nmo, nmo))
    t[no:, :no] = t1.T  # t[a][i] = t^a_i
    return np.eye(nmo) - t, np.eye(nmo) + t


def transformed_hamiltonian(eps, L, t1):
    """Full (nmo)^4 integrals and Fock matrix in the T1-transformed basis.

    g_pqrs = sum_J L^J_pq L^J_rs; h from F^HF = h + sum_l (2 g_pqll - g_pllq) = diag(eps);
    every index of h and g transformed with (1 - t) on the left and (1 + t) on the right.
    """
    no = t1.shape[0]
    nmo = L.shape[1]
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    o = slice(0, no)
    h = np.diag(eps) - (2.0 * np.einsum("pqll->pq", g[:, :, o, o])
                        - np.einsum("pllq->pq", g[:, o, o, :]))
    left, right = _t1_matrices(t1, nmo)
    ht = left @ h @ right
    gt = np.einsum("pP,qQ,rR,sS,PQRS->pqrs", left, right.T, left, right.T, g, optimize=True)
    Ft = ht + 2.0 * np.einsum("pqll->pq", gt[:, :, o, o]) - np.einsum("pllq->pq", gt[:, o, o, :])
    return gt, Ft


def residual_bruteforce(eps, L, t1, t2):
    """(Omega1, Omega2, tau_full) by the plain definition over all ordered triples."""
    tt, tau, g_ovov, g_ooov, g_vvov, F = _full_contravariant(eps, L, t1, t2)
    O1 = np.einsum("ijkabc,jbkc->ia", tt, g_ovov, optimize=True)
    O2 = (np.einsum("ijkabc,kc->ijab", tt, F, optimize=True)
          - np.einsum("ijkabc,jlkc->ilab", tt, g_ooov, optimize=True)
          + np.einsum("ijkabc,dbkc->ijad", tt, g_vvov, optimize=True))
    Y = 2.0 * O2 + O2.transpose(0, 1, 3, 2)
    return O1, (Y + Y.transpose(1, 0, 3, 2)) / 3.0, tau


def jacobian_prep_bruteforce(eps, L, t1, t2):
    """The intermediates of the preparation for the Jacobian transformations by their
    plain definition over all ordered triples (j, k summed freely):
        Zv[a][b][i][d] = - sum_{jkc} tau~^{abc}_{ijk} g_{jdkc}
        Zo[a][j][i][l] =   sum_{kbc} tau~^{abc}_{ijk} g_{lbkc}"""
    tt, _, g_ovov, _, _, _ = _full_contravariant(eps, L, t1, t2)
    Zv = -np.einsum("ijkabc,jdkc->abid", tt, g_ovov, optimize=True)
    Zo = np.einsum("ijkabc,lbkc->ajil", tt, g_ovov, optimize=True)
    return Zv, Zo


def _full_contravariant(eps, L, t1, t2):
    """tau~ and tau over all ordered triples, with the blocks their contractions use."""
    no, _, nv, _ = t2.shape
    gt, Ft = transformed_hamiltonian(eps, L, t1)
    o, v = slice(0, no), slice(no, None)
    g_vvvo = gt[v, v, v, o]
    g_oovo = gt[o, o, v, o]
    g_ovov = gt[o, v, o, v]
    g_ooov = gt[o, o, o, v]
    g_vvov = gt[v, v, o, v]
    F = Ft[o, v]
    # W^{abc}_{ijk} for every ordered (i,j,k)
    W = (np.einsum("ijad,bdck->ijkabc", t2, g_vvvo, optimize=True)
         - np.einsum("ilab,ljck->ijkabc", t2, g_oovo, optimize=True))
    # simultaneous permutations of (a,i), (b,j), (c,k)
    X = (W + np.einsum("jikbac->ijkabc", W) + np.einsum("kjicba->ijkabc", W)
         + np.einsum("ikjacb->ijkabc", W) + np.einsum("jkibca->ijkabc", W)
         + np.einsum("kijcab->ijkabc", W))
    eo, ev = eps[:no], eps[no:]
    D = (ev[None, None, None, :, None, None] + ev[None, None, None, None, :, None]
         + ev[None, None, None, None, None, :] - eo[:, None, None, None, None, None]
         - eo[None, :, None, None, None, None] - eo[None, None, :, None, None, None])
    tau = -X / D
    tt = (4.0 * tau - 2.0 * np.einsum("ijkacb->ijkabc", tau) - 2.0 * np.einsum("ijkcba->ijkabc", tau)
          - 2.0 * np.einsum("ijkbac->ijkabc", tau) + np.einsum("ijkbca->ijkabc", tau)
          + np.einsum("ijkcab->ijkabc", tau))
    return tt, tau, g_ovov, g_ooov, g_vvov, F


def _simultaneous_p(W):
    """P^{abc}_{ijk}: the sum over the six simultaneous permutations of (a,i), (b,j), (c,k)."""
    return (W + np.einsum("jikbac->ijkabc", W) + np.einsum("kjicba->ijkabc", W)
            + np.einsum("ikjacb->ijkabc", W) + np.einsum("jkibca->ijkabc", W)
            + np.einsum("kijcab->ijkabc", W))


def _virtual_contravariant(x):
    return (4.0 * x - 2.0 * np.einsum("ijkacb->ijkabc", x) - 2.0 * np.einsum("ijkcba->ijkabc", x)
            - 2.0 * np.einsum("ijkbac->ijkabc", x) + np.einsum("ijkbca->ijkabc", x)
            + np.einsum("ijkcab->ijkabc", x))


def transition_density_bruteforce(eps, L, t1, t2, l1, l2, omega):
    """The triples contributions to D^{m,0} by their plain definition over all ordered
    index tuples, with full T3 and L3 tensors:
        L^{abc}_{ijk} = (omega - eps^{abc}_{ijk})^{-1} P^{abc}_{ijk} (L^a_i g_{jbkc}
                        + L^{ab}_{ij} F_{kc} + sum_d L^{ad}_{jk} g_{ibdc} - sum_l L^{ab}_{lk} g_{iljc})
        D_cd = 1/2 sum L~^{abc}_{ijk} t^{abd}_{ijk}       D_kc = sum L^{ab}_{ij} t~^{abc}_{ijk}
        Y^o_{clik} = sum_{jab} L~^{abc}_{ijk} t^{ab}_{lj}  D_ld = - sum_{cik} Y^o_{clik} t^{cd}_{ki}
        D_lk = - 1/2 sum L~^{abc}_{ijk} t^{abc}_{ijl}
    Returns (D_cd, D_kc, D_ld, D_lk, Y^o)."""
    no, _, nv, _ = t2.shape
    tt, tau, _, _, _, _ = _full_contravariant(eps, L, t1, t2)
    gt, Ft = transformed_hamiltonian(eps, L, t1)
    o, v = slice(0, no), slice(no, None)
    g_ovov, g_ovvv, g_ooov, F = gt[o, v, o, v], gt[o, v, v, v], gt[o, o, o, v], Ft[o, v]
    C = (np.einsum("ia,jbkc->ijkabc", l1, g_ovov, optimize=True)
         + np.einsum("ijab,kc->ijkabc", l2, F, optimize=True)
         + np.einsum("jkad,ibdc->ijkabc", l2, g_ovvv, optimize=True)
         - np.einsum("lkab,iljc->ijkabc", l2, g_ooov, optimize=True))
    eo, ev = eps[:no], eps[no:]
    D = (ev[None, None, None, :, None, None] + ev[None, None, None, None, :, None]
         + ev[None, None, None, None, None, :] - eo[:, None, None, None, None, None]
         - eo[None, :, None, None, None, None] - eo[None, None, :, None, None, None])
    lam = _simultaneous_p(C) / (omega - D)
    lt = _virtual_contravariant(lam)
    D_cd = 0.5 * np.einsum("ijkabc,ijkabd->cd", lt, tau, optimize=True)
    D_kc = np.einsum("ijab,ijkabc->kc", l2, tt, optimize=True)
    Y = np.einsum("ijkabc,ljab->clik", lt, t2, optimize=True)
    D_ld = -np.einsum("clik,kicd->ld", Y, t2, optimize=True)
    D_lk = -0.5 * np.einsum("ijkabc,ijlabc->lk", lt, tau, optimize=True)
    return D_cd, D_kc, D_ld, D_lk, Y
