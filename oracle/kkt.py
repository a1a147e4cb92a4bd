"""Dense / sparse FP64 references that pin the oracle (test infrastructure only).

Everything here is a plain definition written out with library primitives, so that it
can be checked against MPCGPU Section III by eye:

* ``assemble``      -- G, g, C, c of the KKT system (Section III-A, eq. (4)).
* ``kkt_solve``     -- [G C^T; C 0][-dZ; lambda] = [g; c] solved by LU (O1): the exact
                       solution the iterative method approximates.
* ``schur_dense``   -- S = C G^-1 C^T and gamma = C G^-1 g - c as sparse/dense products
                       (eq. (5), both sides negated so that S is positive definite).
* ``riccati``       -- textbook discrete-time LQR recursion (cost-to-go V_k(x) =
                       1/2 x^T P_k x + p_k^T x); its costate P_k x_k + p_k is lambda_k.
* ``banded_solve``  -- lambda from a banded Cholesky solve of S (scipy.linalg.solveh_banded).
* ``adjoint_dense`` -- gradients of a scalar loss through the KKT solve (O4), from
                       dL/db = nu and dL/dK = -nu w^T with K nu = dL/dw.
* ``autograd_grads``-- the same gradients by torch FP64 autograd through a dense solve.

N state knots x_0..x_{N-1}, N-1 controls; the input x0 is the required dx_0, so
c_0 = -x0; e_k are the dynamics defects (c_{k+1} = e_k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _f64(prob):
    P = {k: np.asarray(v, dtype=np.float64) for k, v in prob.items() if k in
         ("Q", "R", "A", "B", "q", "r", "x0", "e")}
    N, nx = P["q"].shape
    nu = P["R"].shape[-1]
    if "e" not in P or P["e"].size == 0:
        P["e"] = np.zeros((N - 1, nx))
    return P, N, nx, nu


def _offsets(N, nx, nu):
    """Column offset of x_k and u_k in z = [x_0, u_0, x_1, ..., x_{N-1}]."""
    xo = [k * (nx + nu) for k in range(N)]
    uo = [k * (nx + nu) + nx for k in range(N - 1)]
    return xo, uo


def assemble(prob, sparse=False):
    """G, g, C, c of the KKT system (Section III-A)."""
    P, N, nx, nu = _f64(prob)
    nz = N * nx + (N - 1) * nu
    nl = N * nx
    xo, uo = _offsets(N, nx, nu)
    G = sp.lil_matrix((nz, nz))
    g = np.zeros(nz)
    for k in range(N):
        G[xo[k]:xo[k] + nx, xo[k]:xo[k] + nx] = P["Q"][k]
        g[xo[k]:xo[k] + nx] = P["q"][k]
    for k in range(N - 1):
        G[uo[k]:uo[k] + nu, uo[k]:uo[k] + nu] = P["R"][k]
        g[uo[k]:uo[k] + nu] = P["r"][k]
    Cm = sp.lil_matrix((nl, nz))
    c = np.zeros(nl)
    Cm[0:nx, xo[0]:xo[0] + nx] = np.eye(nx)
    c[0:nx] = -P["x0"]
    for k in range(N - 1):
        row = (k + 1) * nx
        Cm[row:row + nx, xo[k]:xo[k] + nx] = -P["A"][k]
        Cm[row:row + nx, uo[k]:uo[k] + nu] = -P["B"][k]
        Cm[row:row + nx, xo[k + 1]:xo[k + 1] + nx] = np.eye(nx)
        c[row:row + nx] = P["e"][k]
    if sparse:
        return G.tocsc(), g, Cm.tocsc(), c
    return G.toarray(), g, Cm.toarray(), c


def _split_z(z, N, nx, nu):
    xo, uo = _offsets(N, nx, nu)
    dx = np.stack([z[o:o + nx] for o in xo])
    du = np.stack([z[o:o + nu] for o in uo]) if N > 1 else np.zeros((0, nu))
    return dx, du


def kkt_matrix(prob, sparse=False):
    G, g, Cm, c = assemble(prob, sparse=sparse)
    if sparse:
        K = sp.bmat([[G, Cm.T], [Cm, None]], format="csc")
    else:
        nl = Cm.shape[0]
        K = np.block([[G, Cm.T], [Cm, np.zeros((nl, nl))]])
    return K, np.concatenate([g, c])


def primal_step(prob, lam):
    """The primal step of a given multiplier: dZ = -G^-1 (g - C^T lambda) (Section III-B),
    by a sparse solve with the block-diagonal G.  Returns (dx [N, nx], du [N-1, nu])."""
    P, N, nx, nu = _f64(prob)
    G, g, Cm, _ = assemble(prob, sparse=True)
    rhs = g - Cm.T @ np.asarray(lam, dtype=np.float64).ravel()
    dZ = -spla.spsolve(G, rhs)
    return _split_z(dZ, N, nx, nu)


def kkt_solve(prob, sparse=None):
    """Exact (lambda, dx, du) from the KKT system by LU; dense LAPACK for small systems,
    SuperLU on the sparse matrix for large ones."""
    P, N, nx, nu = _f64(prob)
    nz = N * nx + (N - 1) * nu
    if sparse is None:
        sparse = nz + N * nx > 2500
    K, b = kkt_matrix(prob, sparse=sparse)
    w = spla.spsolve(K, b) if sparse else np.linalg.solve(K, b)
    dZ = -w[:nz]
    lam = w[nz:].reshape(N, nx)
    dx, du = _split_z(dZ, N, nx, nu)
    return dict(lam=lam, dx=dx, du=du)


def schur_dense(prob):
    """S = C G^-1 C^T ([N*nx, N*nx] dense) and gamma = C G^-1 g - c ([N, nx])."""
    P, N, nx, nu = _f64(prob)
    G, g, Cm, c = assemble(prob, sparse=True)
    Gi = spla.inv(G.tocsc())
    S = (Cm @ Gi @ Cm.T).toarray()
    gam = Cm @ (Gi @ g) - c
    return S, gam.reshape(N, nx)


def blocks_to_dense(M):
    """[N,3,nx,nx] block-tridiagonal storage -> dense [N*nx, N*nx]."""
    N, _, nx, _ = M.shape
    D = np.zeros((N * nx, N * nx))
    for b in range(N):
        for slot in range(3):
            cidx = b + slot - 1
            if 0 <= cidx < N:
                D[b * nx:(b + 1) * nx, cidx * nx:(cidx + 1) * nx] = M[b, slot]
    return D


def riccati(prob):
    """Textbook LQR backward recursion + forward rollout (independent of the KKT/Schur
    route).  Dynamics dx_{k+1} = A_k dx_k + B_k du_k - e_k, dx_0 = x0.
    Returns dict(lam, dx, du) with the costate lambda_k = P_k dx_k + p_k."""
    P, N, nx, nu = _f64(prob)
    Pm = [None] * N
    pv = [None] * N
    Kf = [None] * (N - 1)
    kf = [None] * (N - 1)
    Pm[N - 1] = P["Q"][N - 1].copy()
    pv[N - 1] = P["q"][N - 1].copy()
    for k in range(N - 2, -1, -1):
        A, B, d = P["A"][k], P["B"][k], -P["e"][k]
        Pn, pn = Pm[k + 1], pv[k + 1]
        h = Pn @ d + pn
        Quu = P["R"][k] + B.T @ Pn @ B
        Qux = B.T @ Pn @ A
        Qxx = P["Q"][k] + A.T @ Pn @ A
        Qu = P["r"][k] + B.T @ h
        Qx = P["q"][k] + A.T @ h
        Kf[k] = -np.linalg.solve(Quu, Qux)
        kf[k] = -np.linalg.solve(Quu, Qu)
        Pm[k] = Qxx + Qux.T @ Kf[k]
        Pm[k] = 0.5 * (Pm[k] + Pm[k].T)
        pv[k] = Qx + Qux.T @ kf[k]
    dx = np.zeros((N, nx))
    du = np.zeros((N - 1, nu))
    dx[0] = P["x0"]
    for k in range(N - 1):
        du[k] = Kf[k] @ dx[k] + kf[k]
        dx[k + 1] = P["A"][k] @ dx[k] + P["B"][k] @ du[k] - P["e"][k]
    lam = np.stack([Pm[k] @ dx[k] + pv[k] for k in range(N)])
    return dict(lam=lam, dx=dx, du=du)


def banded_solve(S_blocks, gamma):
    """lambda = S^-1 gamma by banded Cholesky (LAPACK pbsv via scipy), S given in the
    [N,3,nx,nx] block storage.  Lower bandwidth of S is 2*nx-1."""
    N, _, nx, _ = S_blocks.shape
    n = N * nx
    u = 2 * nx - 1
    ab = np.zeros((u + 1, n))          # upper form: ab[u + i - j, j] = S[i, j], i <= j
    for b in range(N):
        for slot in (1, 2):
            cb = b + slot - 1
            if cb >= N:
                continue
            blk = S_blocks[b, slot]
            for ii in range(nx):
                i = b * nx + ii
                for jj in range(nx):
                    j = cb * nx + jj
                    if i <= j and j - i <= u:
                        ab[u + i - j, j] = blk[ii, jj]
    lam = sla.solveh_banded(ab, np.asarray(gamma, dtype=np.float64).ravel(), lower=False)
    return lam.reshape(N, nx)


def adjoint_dense(prob, gl, gx=None, gu=None):
    """Gradients of L(lambda, dx, du) with dL/dlambda = gl, dL/ddx = gx, dL/ddu = gu,
    by the adjoint of the dense KKT solve (O4).

    K w = b with w = [-dZ; lambda], b = [g; c].  The adjoint nu solves K^T nu = dL/dw =
    [-gz; gl]; then dL/db = nu and dL/dK = -nu w^T.  K holds G (top-left), C^T (top-right)
    and C (bottom-left), so dL/dG = -nu1 w1^T and dL/dC = -nu2 w1^T - w2 nu1^T.  Inputs map
    as G(x_k,x_k) = Q_k, G(u_k,u_k) = R_k, C(k+1, x_k) = -A_k, C(k+1, u_k) = -B_k,
    g = [q_0, r_0, ...], c_0 = -x0, c_{k+1} = e_k.  Symmetric Q, R get the symmetric part.
    """
    P, N, nx, nu = _f64(prob)
    nz = N * nx + (N - 1) * nu
    K, b = kkt_matrix(prob, sparse=False)
    w = np.linalg.solve(K, b)
    gz = np.zeros(nz)
    xo, uo = _offsets(N, nx, nu)
    if gx is not None:
        for k in range(N):
            gz[xo[k]:xo[k] + nx] = gx[k]
    if gu is not None:
        for k in range(N - 1):
            gz[uo[k]:uo[k] + nu] = gu[k]
    dLdw = np.concatenate([-gz, np.asarray(gl, dtype=np.float64).ravel()])
    nu_ = np.linalg.solve(K.T, dLdw)
    n1, n2 = nu_[:nz], nu_[nz:]
    w1, w2 = w[:nz], w[nz:]
    dG = -np.outer(n1, w1)
    dC = -np.outer(n2, w1) - np.outer(w2, n1)
    sym = lambda M: 0.5 * (M + M.T)
    out = dict(
        dQ=np.stack([sym(dG[xo[k]:xo[k] + nx, xo[k]:xo[k] + nx]) for k in range(N)]),
        dR=np.stack([sym(dG[uo[k]:uo[k] + nu, uo[k]:uo[k] + nu]) for k in range(N - 1)])
        if N > 1 else np.zeros((0, nu, nu)),
        dA=np.stack([-dC[(k + 1) * nx:(k + 2) * nx, xo[k]:xo[k] + nx] for k in range(N - 1)])
        if N > 1 else np.zeros((0, nx, nx)),
        dB=np.stack([-dC[(k + 1) * nx:(k + 2) * nx, uo[k]:uo[k] + nu] for k in range(N - 1)])
        if N > 1 else np.zeros((0, nx, nu)),
        dq=np.stack([n1[xo[k]:xo[k] + nx] for k in range(N)]),
        dr=np.stack([n1[uo[k]:uo[k] + nu] for k in range(N - 1)]) if N > 1 else np.zeros((0, nu)),
        dx0=-n2[0:nx].copy(),
        de=np.stack([n2[(k + 1) * nx:(k + 2) * nx] for k in range(N - 1)])
        if N > 1 else np.zeros((0, nx)),
    )
    return out


def autograd_grads(prob, loss="lam_sq"):
    """Gradients of L = ||lambda||^2 by torch FP64 autograd through a dense KKT solve
    (a third, independent route).  Symmetric inputs get the symmetric part."""
    import torch

    P, N, nx, nu = _f64(prob)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    nz = N * nx + (N - 1) * nu
    nl = N * nx
    xo, uo = _offsets(N, nx, nu)
    K = torch.zeros((nz + nl, nz + nl), dtype=torch.float64)
    b = torch.zeros(nz + nl, dtype=torch.float64)
    # build K and b with index_put so gradients flow to every input block
    Kl = K.clone()
    for k in range(N):
        Kl = Kl.index_put((torch.arange(xo[k], xo[k] + nx)[:, None],
                           torch.arange(xo[k], xo[k] + nx)[None, :]), T["Q"][k])
        b = b.index_put((torch.arange(xo[k], xo[k] + nx),), T["q"][k])
    for k in range(N - 1):
        Kl = Kl.index_put((torch.arange(uo[k], uo[k] + nu)[:, None],
                           torch.arange(uo[k], uo[k] + nu)[None, :]), T["R"][k])
        b = b.index_put((torch.arange(uo[k], uo[k] + nu),), T["r"][k])
    Cm = torch.zeros((nl, nz), dtype=torch.float64)
    Cm = Cm.index_put((torch.arange(0, nx)[:, None], torch.arange(xo[0], xo[0] + nx)[None, :]),
                      torch.eye(nx, dtype=torch.float64))
    cvec = torch.zeros(nl, dtype=torch.float64)
    cvec = cvec.index_put((torch.arange(0, nx),), -T["x0"])
    for k in range(N - 1):
        r0 = (k + 1) * nx
        ri = torch.arange(r0, r0 + nx)[:, None]
        Cm = Cm.index_put((ri, torch.arange(xo[k], xo[k] + nx)[None, :]), -T["A"][k])
        Cm = Cm.index_put((ri, torch.arange(uo[k], uo[k] + nu)[None, :]), -T["B"][k])
        Cm = Cm.index_put((ri, torch.arange(xo[k + 1], xo[k + 1] + nx)[None, :]),
                          torch.eye(nx, dtype=torch.float64))
        cvec = cvec.index_put((torch.arange(r0, r0 + nx),), T["e"][k])
    Kfull = Kl.clone()
    Kfull = Kfull.index_put((torch.arange(nz, nz + nl)[:, None], torch.arange(0, nz)[None, :]), Cm)
    Kfull = Kfull.index_put((torch.arange(0, nz)[:, None], torch.arange(nz, nz + nl)[None, :]), Cm.T)
    bfull = b.index_put((torch.arange(nz, nz + nl),), cvec)
    w = torch.linalg.solve(Kfull, bfull)
    lam = w[nz:]
    if loss != "lam_sq":
        raise ValueError(loss)
    L = (lam * lam).sum()
    L.backward()
    sym = lambda M: 0.5 * (M + M.transpose(-1, -2))
    return dict(dQ=sym(T["Q"].grad).numpy(), dR=sym(T["R"].grad).numpy(), dA=T["A"].grad.numpy(),
                dB=T["B"].grad.numpy(), dq=T["q"].grad.numpy(), dr=T["r"].grad.numpy(),
                dx0=T["x0"].grad.numpy(), de=T["e"].grad.numpy(), lam=lam.detach().numpy().reshape(N, nx))
