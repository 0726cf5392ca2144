"""Dense three-field hybridised system of eq. syslinhyb (Section 3.2), for tiny meshes.

Test infrastructure only.  The matrices A^, D^, C^ and R^ are assembled
literally from H^_K, A_K + E_K, D_K, F_K, C_K and R_K, and the square system

    [ A^  D^t  C^t ] [U^]   [R^]
    [ D^   0    0  ] [P^] = [ 0]
    [ C^   0    0  ] [W^]   [ 0]

is solved by dense LU.  Also builds J = sum H_K H^_K^t (Section 3.2 item 2).
"""
from __future__ import annotations

import numpy as np

from .cr import Problem, element_E, restrict


def three_field(P: Problem, E=None, signs=None):
    m = P.mesh
    d = P.d
    if E is None:
        E = element_E(P)
    if signs is None:
        signs = m.sign
    blocks = []
    off = 0
    for k in range(m.ne):
        Ak, Dk, Rk, gk, idx = restrict(P, k)
        blocks.append((k, Ak + np.diag(E[k][idx]), Dk, Rk, gk, np.repeat(signs[k], d)[idx], off))
        off += len(idx)
    nU = off
    nP = m.ne - 1
    nW = m.nf * d
    prow = {}
    r = 0
    for k in range(m.ne):
        if k != P.k0:
            prow[k] = r
            r += 1
    Ahat = np.zeros((nU, nU))
    Dhat = np.zeros((nP, nU))
    Chat = np.zeros((nW, nU))
    J = np.zeros((nW, nU))
    Rhat = np.zeros(nU)
    for k, Ak, Dk, Rk, gk, ck, o in blocks:
        n = len(gk)
        Ahat[o:o + n, o:o + n] = Ak
        if k != P.k0:
            Dhat[prow[k], o:o + n] = Dk
        Chat[gk, o + np.arange(n)] = ck
        J[gk, o + np.arange(n)] = 1.0
        Rhat[o:o + n] = Rk
    N = nU + nP + nW
    M = np.zeros((N, N))
    M[:nU, :nU] = Ahat
    M[:nU, nU:nU + nP] = Dhat.T
    M[:nU, nU + nP:] = Chat.T
    M[nU:nU + nP, :nU] = Dhat
    M[nU + nP:, :nU] = Chat
    rhs = np.concatenate([Rhat, np.zeros(nP + nW)])
    sol = np.linalg.solve(M, rhs)
    Uhat = sol[:nU]
    Phat = sol[nU:nU + nP]
    What = sol[nU + nP:]
    Pk = np.zeros(m.ne)
    for k, rr in prow.items():
        Pk[k] = Phat[rr]
    # the common value of the two copies, read from the C = +1 copy
    U = np.zeros(nW)
    for k, Ak, Dk, Rk, gk, ck, o in blocks:
        own = ck > 0
        U[gk[own]] = Uhat[o:o + len(gk)][own]
    return dict(M=M, Ahat=Ahat, Dhat=Dhat, Chat=Chat, J=J, Rhat=Rhat, Uhat=Uhat, P=Pk,
                W=What, U=U.reshape(-1, d), blocks=blocks, size=(nU, nP, nW))
