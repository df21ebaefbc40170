"""Brute-force evaluation of the CC3 triples residual (and of the t3-dependent
intermediates of the Jacobian preparation) over the full T3 tensor.

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
