"""Plain FP64 CPU oracle of the 3-D (hexahedral) vertex-patch multigrid.

TEST INFRASTRUCTURE ONLY: imported by tests/.  The product library never imports,
links or runs anything here, and nothing here calls the library.

It follows the method's definitions as written, for d = 3:
  * discretisation (Section 2): RT_k x dQ_k on a uniform hexahedral mesh of the unit
    cube, the interior-penalty Brinkman form (eq. ipbrinkman) with sigma_h = sigma / h,
    pressure coupling -(p, div v) - (q, div u) (eq. Brinkman-weak); on a Dirichlet
    side the normal velocity is essential (boundary normal face dofs fixed to the face
    projection of g.n, identity rows and columns, lifting into the right-hand side) and
    the tangential velocity is imposed by the Nitsche terms of eq. (BCh) (the reading
    the two-dimensional path takes: with a weak normal component the form misses
    <p, v.n> and the polynomial patch test fails); an open side carries the natural
    condition mu d_n u - p n = 0 (no boundary term, no data); with every side
    Dirichlet the pressure is taken in L2_0;
  * mesh hierarchy (Section 3): N_j = N_0 2^j, kappa of a coarse cell = mean of its
    eight children (the arithmetic average used in the experiments);
  * transfers (Section 3): the exact embedding of the nested coarse space, computed
    per fine cell as the local L2 projection of the parent's basis functions (exact,
    since the coarse function lies in the fine cell's local space) and assigned per
    fine dof; restriction is its transpose;
  * smoother (Section 3): vertex patches of up to eight cells (each cell lies in at
    most eight patches in 3-D), S = dofs whose support lies in the patch cells,
    local Ritz projection through the patch pseudo-inverse (a patch without a free
    boundary normal dof, i.e. one not touching an open side, has the patch-constant
    pressure in its kernel), symmetric
    multiplicative sweep over 27 colours (vx mod 3) + 3 (vy mod 3) + 9 (vz mod 3),
    order 0..26, 25..0;
  * V-cycle with the coarse-grid correction x += P B_{j-1} P^T (b - A x), variable
    smoothing m_j = m_J 2^(J-j) (or fixed), exact coarse solve (bordered with the
    constant pressure when every side is Dirichlet), identity rows of the essential dofs inverted exactly; right-preconditioned
    FGMRES with modified Gram-Schmidt (the Krylov method of the experiments).
Integrals use Gauss-Legendre rules with k + 2 points per direction, exact for every
integrand here (cellwise constant kappa, polynomial data of low degree).

Numbering (a specification the library follows in code of its own):
  NB = k + 1; cells c = (cz N + cy) N + cx; h = 1 / N.
  velocity component d in {0, 1, 2}, transverse axes (d1, d2) = the other two in
  increasing order; basis psi_a(xi_d) L_b(xi_d1) L_c(xi_d2), a = 0 .. k+1, b, c = 0 .. k,
  with psi_0 = 1 - t, psi_1 = t, psi_a = int_0^t L_{a-1} (a >= 2) and L_b the
  orthonormal Legendre polynomials on [0, 1];
  face dofs (a = 0 / 1: the face at cell index i = c_d / c_d + 1 along d):
      d NF + ((t2 N + t1)(N + 1) + i) NB^2 + b + NB c,   NF = (N + 1) N^2 NB^2,
      (t1, t2) = the cell indices along d1, d2;
  interior dofs (a >= 2): 3 NF + c NI + (d k + a - 2) NB^2 + b + NB c, NI = 3 k NB^2;
  pressure L_a(x) L_b(y) L_c(z): n_u + c NB^3 + a + NB b + NB^2 c.
Sides: bc[s] for s = 2 d + (0 at x_d = 0, 1 at x_d = 1), 0 Dirichlet, 1 open.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import Polynomial as Poly
from numpy.polynomial import legendre as npleg

AXES = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


# ---------------------------------------------------------------- 1-D functions
def legendre01(b: int) -> Poly:
    """Orthonormal Legendre polynomial of degree b on [0, 1]."""
    c = np.zeros(b + 1)
    c[b] = 1.0
    return np.sqrt(2 * b + 1) * Poly(npleg.leg2poly(c))(Poly([-1.0, 2.0]))


def psi(a: int) -> Poly:
    """psi_0 = 1 - t, psi_1 = t, psi_a = int_0^t L_{a-1} (a >= 2)."""
    if a == 0:
        return Poly([1.0, -1.0])
    if a == 1:
        return Poly([0.0, 1.0])
    return legendre01(a - 1).integ(lbnd=0)


def gauss01(q: int):
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


# ---------------------------------------------------------------- discretisation
DIRICHLET = (0, 0, 0, 0, 0, 0)


class Space:
    """Sizes and the dof numbering of one level (N cells per side, degree k, sides bc)."""

    def __init__(self, N: int, k: int, bc=DIRICHLET):
        self.N, self.k, self.NB = N, k, k + 1
        self.bc = tuple(int(v) for v in bc)
        NB = self.NB
        self.NF = (N + 1) * N * N * NB * NB
        self.NI = 3 * k * NB * NB
        self.n_u = 3 * self.NF + N ** 3 * self.NI
        self.n_p = N ** 3 * NB ** 3
        self.ndof = self.n_u + self.n_p
        # local velocity dofs (d, a, b, c) and pressure dofs (a, b, c)
        self.lu = [(d, a, b, c) for d in range(3) for a in range(k + 2) for c in range(NB) for b in range(NB)]
        self.lp = [(a, b, c) for c in range(NB) for b in range(NB) for a in range(NB)]
        # essential dofs: the normal face dofs on the boundary faces (i = 0 or N) of the
        # Dirichlet sides; the normal face dofs of the open sides are free
        self.cons = np.zeros(self.ndof, dtype=bool)
        self.open_normal = np.zeros(self.ndof, dtype=bool)
        for d in range(3):
            for t2 in range(N):
                for t1 in range(N):
                    for side, i in ((0, 0), (1, N)):
                        base = d * self.NF + ((t2 * N + t1) * (N + 1) + i) * NB * NB
                        mask = self.open_normal if self.bc[2 * d + side] else self.cons
                        mask[base:base + NB * NB] = True
        self.all_dirichlet = not any(self.bc)

    def cell(self, cx, cy, cz):
        return (cz * self.N + cy) * self.N + cx

    def gu(self, cc, d, a, b, c):
        """Global index of local velocity dof (d, a, b, c) of cell cc = (cx, cy, cz)."""
        N, NB = self.N, self.NB
        if a <= 1:
            d1, d2 = AXES[d]
            i = cc[d] + a
            return d * self.NF + ((cc[d2] * N + cc[d1]) * (N + 1) + i) * NB * NB + b + NB * c
        return 3 * self.NF + self.cell(*cc) * self.NI + (d * self.k + a - 2) * NB * NB + b + NB * c

    def gp(self, cc, a, b, c):
        NB = self.NB
        return self.n_u + self.cell(*cc) * NB ** 3 + a + NB * b + NB * NB * c

    def cell_dofs(self, cc):
        return np.array([self.gu(cc, *t) for t in self.lu] + [self.gp(cc, *t) for t in self.lp], dtype=np.int64)


class RefBasis:
    """Local basis on the reference cube [0, 1]^3 (values, gradients, divergence)."""

    def __init__(self, k: int):
        self.k = k
        NB = k + 1
        self.L = [legendre01(b) for b in range(NB)]
        self.P = [psi(a) for a in range(k + 2)]
        self.lu = [(d, a, b, c) for d in range(3) for a in range(k + 2) for c in range(NB) for b in range(NB)]
        self.lp = [(a, b, c) for c in range(NB) for b in range(NB) for a in range(NB)]

    def vel(self, X):
        """X: (n, 3) points.  Returns val (nu, n, 3), grad (nu, n, 3, 3) [comp, deriv]."""
        n = X.shape[0]
        nu = len(self.lu)
        val = np.zeros((nu, n, 3))
        grad = np.zeros((nu, n, 3, 3))
        for i, (d, a, b, c) in enumerate(self.lu):
            d1, d2 = AXES[d]
            fa, fb, fc = self.P[a], self.L[b], self.L[c]
            va, vb, vc = fa(X[:, d]), fb(X[:, d1]), fc(X[:, d2])
            val[i, :, d] = va * vb * vc
            grad[i, :, d, d] = fa.deriv()(X[:, d]) * vb * vc
            grad[i, :, d, d1] = va * fb.deriv()(X[:, d1]) * vc
            grad[i, :, d, d2] = va * vb * fc.deriv()(X[:, d2])
        return val, grad

    def pres(self, X):
        return np.array([self.L[a](X[:, 0]) * self.L[b](X[:, 1]) * self.L[c](X[:, 2]) for (a, b, c) in self.lp])


def cube_rule(q):
    x, w = gauss01(q)
    X = np.array([(x[i], x[j], x[l]) for l in range(q) for j in range(q) for i in range(q)])
    W = np.array([w[i] * w[j] * w[l] for l in range(q) for j in range(q) for i in range(q)])
    return X, W


def face_rule(q, d, xi_d):
    """Points on the face xi_d = const of the reference cube, and weights."""
    x, w = gauss01(q)
    d1, d2 = AXES[d]
    X = np.zeros((q * q, 3))
    W = np.zeros(q * q)
    for j in range(q):
        for i in range(q):
            X[j * q + i, d] = xi_d
            X[j * q + i, d1] = x[i]
            X[j * q + i, d2] = x[j]
            W[j * q + i] = w[i] * w[j]
    return X, W


class Level:
    """Assembled FP64 operator of one level (CSR), with its reference matrices."""

    def __init__(self, N, k, mu, sigma, kappa, bc=DIRICHLET):
        self.sp = S = Space(N, k, bc)
        self.N, self.k, self.mu, self.sigma = N, k, mu, sigma
        self.kappa = np.asarray(kappa, dtype=np.float64).reshape(N ** 3)
        h = 1.0 / N
        self.h = h
        rb = RefBasis(k)
        self.rb = rb
        q = k + 2
        X, W = cube_rule(q)
        v, g = rb.vel(X)
        pv = rb.pres(X)
        div = np.einsum("inkk->in", g)
        # cell integrals on a cell of size h: grad = ghat / h, volume h^3
        Kc = mu * h * np.einsum("iqab,jqab,q->ij", g, g, W)
        Mc = h ** 3 * np.einsum("iqa,jqa,q->ij", v, v, W)
        Bc = -h ** 2 * np.einsum("pq,iq,q->pi", pv, div, W)
        nu, npl = len(rb.lu), len(rb.lp)
        rows, cols, vals = [], [], []
        cells = [(cx, cy, cz) for cz in range(N) for cy in range(N) for cx in range(N)]
        dofs = np.array([S.cell_dofs(cc) for cc in cells])  # (ncell, nu + np)
        self.cell_dof_table = dofs
        du, dp = dofs[:, :nu], dofs[:, nu:]
        for t in range(len(cells)):
            Auu = Kc + self.kappa[t] * Mc
            rows.append(np.repeat(du[t], nu)); cols.append(np.tile(du[t], nu)); vals.append(Auu.ravel())
            rows.append(np.repeat(dp[t], nu)); cols.append(np.tile(du[t], npl)); vals.append(Bc.ravel())
            rows.append(np.repeat(du[t], npl)); cols.append(np.tile(dp[t], nu)); vals.append(Bc.T.ravel())
        # faces: interior (T1 lower, T2 upper along d, n = e_d) and boundary (n outward)
        pen = 2.0 * mu * sigma / h
        for d in range(3):
            X1, Wf = face_rule(q, d, 1.0)
            X2, _ = face_rule(q, d, 0.0)
            v1, g1 = rb.vel(X1)
            v2, g2 = rb.vel(X2)
            dn1, dn2 = g1[:, :, :, d] / h, g2[:, :, :, d] / h  # (nu, nq, comp): d u / d x_d
            area = h * h
            # [u] = u1 - u2 over the stacked local dofs of T1 then T2
            jmp = np.concatenate([v1, -v2], axis=0)
            avg = 0.5 * np.concatenate([dn1, dn2], axis=0)
            F = area * (pen * np.einsum("iqa,jqa,q->ij", jmp, jmp, Wf)
                        - mu * np.einsum("jqa,iqa,q->ij", avg, jmp, Wf)
                        - mu * np.einsum("iqa,jqa,q->ij", avg, jmp, Wf))
            for side, (Xb, sgn) in enumerate(((X2, -1.0), (X1, 1.0))):
                vb, gb = rb.vel(Xb)
                dnb = sgn * gb[:, :, :, d] / h
                Fb = area * (pen * np.einsum("iqa,jqa,q->ij", vb, vb, Wf)
                             - mu * np.einsum("jqa,iqa,q->ij", dnb, vb, Wf)
                             - mu * np.einsum("iqa,jqa,q->ij", dnb, vb, Wf))
                if side == 0:
                    Fb_lo = Fb
                else:
                    Fb_hi = Fb
            for cc in cells:
                t = S.cell(*cc)
                if cc[d] + 1 < N:
                    up = list(cc)
                    up[d] += 1
                    t2 = S.cell(*up)
                    gl = np.concatenate([du[t], du[t2]])
                    rows.append(np.repeat(gl, 2 * nu)); cols.append(np.tile(gl, 2 * nu)); vals.append(F.ravel())
                # Nitsche terms on Dirichlet sides only (an open side has no boundary term)
                if cc[d] == 0 and not S.bc[2 * d]:
                    rows.append(np.repeat(du[t], nu)); cols.append(np.tile(du[t], nu)); vals.append(Fb_lo.ravel())
                if cc[d] == N - 1 and not S.bc[2 * d + 1]:
                    rows.append(np.repeat(du[t], nu)); cols.append(np.tile(du[t], nu)); vals.append(Fb_hi.ravel())
        r = np.concatenate(rows); c_ = np.concatenate(cols); vv = np.concatenate(vals)
        A = sp.csr_matrix((vv, (r, c_)), shape=(S.ndof, S.ndof))
        A.sum_duplicates()
        A.eliminate_zeros()
        self.A_full = A
        # essential dofs: identity rows and columns
        free = sp.diags((~S.cons).astype(float))
        self.A = (free @ A @ free + sp.diags(S.cons.astype(float))).tocsr()
        self.A.eliminate_zeros()
        self.cells = cells
        # the patch-constant / global-constant pressure vector (cell (0,0,0) coefficients)
        self.cvec = np.zeros(S.ndof)
        self.cvec[S.n_u::S.NB ** 3] = 1.0

    def rhs(self, f, g):
        """F(v, q) = (f, v) + 2 mu sigma_h <g, v>_G - mu <grad v n, g>_G (eq. BCh), G the
        Dirichlet sides (g is never evaluated on an open side); f, g: callables (x, y,
        z arrays) -> (3, n) arrays.  Pressure rows are zero."""
        S, rb, h, mu = self.sp, self.rb, self.h, self.mu
        q = self.k + 2
        X, W = cube_rule(q)
        v, _ = rb.vel(X)
        nu = len(rb.lu)
        b = np.zeros(S.ndof)
        du = self.cell_dof_table[:, :nu]
        for t, cc in enumerate(self.cells):
            P = (np.array(cc)[None, :] + X) * h
            fv = np.asarray(f(P[:, 0], P[:, 1], P[:, 2]), dtype=float)  # (3, nq)
            np.add.at(b, du[t], h ** 3 * np.einsum("iqa,aq,q->i", v, fv, W))
        pen = 2.0 * mu * self.sigma / h
        for d in range(3):
            for side, (xi, sgn) in enumerate(((0.0, -1.0), (1.0, 1.0))):
                if S.bc[2 * d + side]:
                    continue
                Xb, Wf = face_rule(q, d, xi)
                vb, gb = rb.vel(Xb)
                dnb = sgn * gb[:, :, :, d] / h
                for t, cc in enumerate(self.cells):
                    if (xi == 0.0 and cc[d] != 0) or (xi == 1.0 and cc[d] != self.N - 1):
                        continue
                    P = (np.array(cc)[None, :] + Xb) * h
                    gv = np.asarray(g(P[:, 0], P[:, 1], P[:, 2]), dtype=float)
                    np.add.at(b, du[t], h * h * (pen * np.einsum("iqa,aq,q->i", vb, gv, Wf)
                                                 - mu * np.einsum("iqa,aq,q->i", dnb, gv, Wf)))
        gc = self.essential_values(g)
        b = b - self.A_full @ gc
        b[S.cons] = gc[S.cons]
        return b

    def essential_values(self, g):
        """Vector holding, on the essential dofs, the coefficients of the projection of
        g.n onto the face polynomials L_b L_c (orthonormal on a face); zero elsewhere."""
        S, rb, h, N, NB = self.sp, self.rb, self.h, self.N, self.sp.NB
        x, w = gauss01(self.k + 2)
        out = np.zeros(S.ndof)
        for d in range(3):
            d1, d2 = AXES[d]
            for t2 in range(N):
                for t1 in range(N):
                    for side, i in ((0, 0), (1, N)):
                        if S.bc[2 * d + side]:
                            continue
                        base = d * S.NF + ((t2 * N + t1) * (N + 1) + i) * NB * NB
                        for c in range(NB):
                            for b_ in range(NB):
                                acc = 0.0
                                for jj in range(len(x)):
                                    for ii in range(len(x)):
                                        P = np.zeros(3)
                                        P[d] = i * h
                                        P[d1] = (t1 + x[ii]) * h
                                        P[d2] = (t2 + x[jj]) * h
                                        gv = np.asarray(g(P[0:1], P[1:2], P[2:3]), dtype=float)[:, 0]
                                        acc += w[ii] * w[jj] * gv[d] * rb.L[b_](x[ii]) * rb.L[c](x[jj])
                                out[base + b_ + NB * c] = acc
        return out

    def interpolate_pressure(self, p):
        """Coefficients of the L2 projection of the scalar function p onto dQ_k."""
        S, rb, h = self.sp, self.rb, self.h
        X, W = cube_rule(self.k + 2)
        pv = rb.pres(X)
        Mp = np.einsum("pq,rq,q->pr", pv, pv, W)
        out = np.zeros(S.n_p)
        for t, cc in enumerate(self.cells):
            P = (np.array(cc)[None, :] + X) * h
            rhs = np.einsum("pq,q,q->p", pv, p(P[:, 0], P[:, 1], P[:, 2]), W)
            out[t * S.NB ** 3:(t + 1) * S.NB ** 3] = np.linalg.solve(Mp, rhs)
        return out


# ---------------------------------------------------------------- patches
def patch_dofs(S: Space, vx, vy, vz):
    """Sorted dofs of the vertex patch (support inside the patch cells) and its cells."""
    N = S.N
    cells = [(cx, cy, cz) for cz in (vz - 1, vz) for cy in (vy - 1, vy) for cx in (vx - 1, vx)
             if 0 <= cx < N and 0 <= cy < N and 0 <= cz < N]
    cset = set(cells)
    out = set()
    for cc in cells:
        for (d, a, b, c) in S.lu:
            if a <= 1:
                # the face dof is supported by this cell and its neighbour across the face
                nb = list(cc)
                nb[d] += 1 if a == 1 else -1
                if 0 <= nb[d] < N and tuple(nb) not in cset:
                    continue
            gi = S.gu(cc, d, a, b, c)
            if not S.cons[gi]:
                out.add(gi)
        for t in S.lp:
            out.add(S.gp(cc, *t))
    return np.array(sorted(out), dtype=np.int64), cells


def colour_of(vx, vy, vz):
    return (vx % 3) + 3 * (vy % 3) + 9 * (vz % 3)


def patch_pinv(A_S, S: Space, dofs, cells, singular):
    """A_S^+ : the inverse, or for a singular patch (no boundary dof) the leading block
    of the inverse of [[A_S, c], [c^T, 0]], c = normalised patch-constant pressure."""
    n = len(dofs)
    if not singular:
        return np.linalg.inv(A_S)
    c = np.zeros(n)
    pos = {g: i for i, g in enumerate(dofs)}
    for cc in cells:
        c[pos[S.gp(cc, 0, 0, 0)]] = 1.0
    c /= np.linalg.norm(c)
    Bd = np.zeros((n + 1, n + 1))
    Bd[:n, :n] = A_S
    Bd[:n, n] = c
    Bd[n, :n] = c
    return np.linalg.inv(Bd)[:n, :n]


class Smoother:
    """Vertex patches of one level, their pseudo-inverses and the colour lists."""

    def __init__(self, lev: Level):
        S = lev.sp
        N = S.N
        self.lev = lev
        A = lev.A.tocsr()
        self.patches = []
        self.colours = [[] for _ in range(27)]
        for vz in range(N + 1):
            for vy in range(N + 1):
                for vx in range(N + 1):
                    dofs, cells = patch_dofs(S, vx, vy, vz)
                    # without a free boundary normal dof (open sides only) the patch
                    # space has the constant patch pressure in its kernel
                    singular = not S.open_normal[dofs].any()
                    rows = A[dofs, :]
                    A_S = rows[:, dofs].toarray()
                    pinv = patch_pinv(A_S, S, dofs, cells, singular)
                    self.colours[colour_of(vx, vy, vz)].append(len(self.patches))
                    self.patches.append(((vx, vy, vz), dofs, rows.tocsr(), pinv, singular))

    def colour_step(self, col, x, b):
        for pi in self.colours[col]:
            _, dofs, rows, pinv, _ = self.patches[pi]
            r = b[dofs] - rows @ x
            x[dofs] += pinv @ r

    def step(self, x, b):
        """One symmetric multiplicative smoothing step: colours 0..26, 25..0."""
        for col in list(range(27)) + list(range(25, -1, -1)):
            self.colour_step(col, x, b)


# ---------------------------------------------------------------- transfers
def local_transfer(k):
    """T[o] (nloc_f x nloc_c): fine-cell coefficients of the parent's local basis
    functions on the child with offset o = (ox, oy, oz), by local L2 projection."""
    rb = RefBasis(k)
    X, W = cube_rule(k + 2)
    vf, _ = rb.vel(X)
    pf = rb.pres(X)
    Mu = np.einsum("iqa,jqa,q->ij", vf, vf, W)
    Mp = np.einsum("iq,jq,q->ij", pf, pf, W)
    Tu, Tp = {}, {}
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                o = np.array([ox, oy, oz], dtype=float)
                Xc = 0.5 * (o[None, :] + X)
                vc, _ = rb.vel(Xc)
                pc = rb.pres(Xc)
                Tu[(ox, oy, oz)] = np.linalg.solve(Mu, np.einsum("iqa,jqa,q->ij", vf, vc, W))
                Tp[(ox, oy, oz)] = np.linalg.solve(Mp, np.einsum("iq,jq,q->ij", pf, pc, W))
    return Tu, Tp


def prolongation(Sc: Space, Sf: Space):
    """Exact embedding P (n_f x n_c), assigned per fine dof."""
    k = Sc.k
    Tu, Tp = local_transfer(k)
    ent = {}
    Nc = Sc.N
    for cz in range(Nc):
        for cy in range(Nc):
            for cx in range(Nc):
                cdofs = Sc.cell_dofs((cx, cy, cz))
                nu = len(Sc.lu)
                for (ox, oy, oz), T in Tu.items():
                    fc = (2 * cx + ox, 2 * cy + oy, 2 * cz + oz)
                    fdofs = Sf.cell_dofs(fc)
                    Tpp = Tp[(ox, oy, oz)]
                    for i in range(nu):
                        if Sf.cons[fdofs[i]]:
                            continue
                        for j in range(nu):
                            if abs(T[i, j]) > 1e-14 and not Sc.cons[cdofs[j]]:
                                ent.setdefault((fdofs[i], cdofs[j]), T[i, j])
                    for i in range(len(Sc.lp)):
                        for j in range(len(Sc.lp)):
                            if abs(Tpp[i, j]) > 1e-14:
                                ent.setdefault((fdofs[nu + i], cdofs[nu + j]), Tpp[i, j])
    r = np.array([a for a, _ in ent], dtype=np.int64)
    c = np.array([b for _, b in ent], dtype=np.int64)
    v = np.array(list(ent.values()))
    return sp.csr_matrix((v, (r, c)), shape=(Sf.ndof, Sc.ndof))


# ---------------------------------------------------------------- the solver
class Oracle3D:
    def __init__(self, n0, levels, k, mu, sigma, kappa, cycle=1, m_fine=2, bc=DIRICHLET):
        self.k, self.mu, self.sigma = k, mu, sigma
        self.bc = tuple(int(v) for v in bc)
        self.J = levels - 1
        self.cycle, self.m_fine = cycle, m_fine
        Nf = n0 * 2 ** self.J
        kap = [None] * levels
        kap[self.J] = np.asarray(kappa, dtype=np.float64).reshape(Nf, Nf, Nf)  # [cz, cy, cx]
        for j in range(self.J, 0, -1):
            K = kap[j]
            kap[j - 1] = 0.125 * (K[0::2, 0::2, 0::2] + K[1::2, 0::2, 0::2] + K[0::2, 1::2, 0::2] + K[1::2, 1::2, 0::2]
                                  + K[0::2, 0::2, 1::2] + K[1::2, 0::2, 1::2] + K[0::2, 1::2, 1::2]
                                  + K[1::2, 1::2, 1::2])
        self.kap = kap
        self.lev = [Level(n0 * 2 ** j, k, mu, sigma, kap[j].ravel(), self.bc) for j in range(levels)]
        self.sm = [None] + [Smoother(L) for L in self.lev[1:]]
        self.P = [None] + [prolongation(self.lev[j - 1].sp, self.lev[j].sp) for j in range(1, levels)]
        A0 = self.lev[0].A.toarray()
        if self.lev[0].sp.all_dirichlet:
            # the constant pressure spans the kernel: bordered inverse
            c = self.lev[0].cvec / np.linalg.norm(self.lev[0].cvec)
            n0d = A0.shape[0]
            Bd = np.zeros((n0d + 1, n0d + 1))
            Bd[:n0d, :n0d] = A0
            Bd[:n0d, n0d] = c
            Bd[n0d, :n0d] = c
            self.A0inv = np.linalg.inv(Bd)[:n0d, :n0d]
        else:
            self.A0inv = np.linalg.inv(A0)

    def m(self, j):
        return self.m_fine * (2 ** (self.J - j) if self.cycle == 1 else 1)

    def vcycle_level(self, j, b):
        if j == 0:
            return self.A0inv @ b
        A = self.lev[j].A
        x = np.zeros_like(b)
        for _ in range(self.m(j)):
            self.sm[j].step(x, b)
        r = b - A @ x
        x += self.P[j] @ self.vcycle_level(j - 1, self.P[j].T @ r)
        for _ in range(self.m(j)):
            self.sm[j].step(x, b)
        cons = self.lev[j].sp.cons
        x[cons] = b[cons]
        return x

    def vcycle(self, r):
        return self.vcycle_level(self.J, np.asarray(r, dtype=np.float64))

    def apply(self, x, j=None):
        return self.lev[self.J if j is None else j].A @ x

    def direct_solve(self, b):
        """The solution (with zero pressure mean when every side is Dirichlet: bordered
        sparse system)."""
        L = self.lev[self.J]
        if not L.sp.all_dirichlet:
            return spla.spsolve(L.A.tocsc(), b)
        c = L.cvec / np.linalg.norm(L.cvec)
        Bd = sp.bmat([[L.A, sp.csr_matrix(c[:, None])], [sp.csr_matrix(c[None, :]), None]]).tocsc()
        return spla.spsolve(Bd, np.concatenate([b, [0.0]]))[:-1]

    def pressure_mean(self, x, j=None):
        L = self.lev[self.J if j is None else j]
        return x[L.sp.n_u::L.sp.NB ** 3].mean()

    def fgmres(self, b, rtol=1e-10, maxit=200, restart=50, precond=True):
        """Right-preconditioned FGMRES, x0 = 0, modified Gram-Schmidt; stops when the
        Arnoldi residual estimate <= rtol ||b||.  Returns (x, iterations, true rel. res.)."""
        A = self.lev[self.J].A
        n = b.size
        x = np.zeros(n)
        bn = np.linalg.norm(b)
        its = 0
        while its < maxit:
            r = b - A @ x
            beta = np.linalg.norm(r)
            if beta <= rtol * bn:
                break
            m = min(restart, maxit - its)
            V = np.zeros((m + 1, n))
            Z = np.zeros((m, n))
            H = np.zeros((m + 1, m))
            V[0] = r / beta
            g = np.zeros(m + 1)
            g[0] = beta
            cs, sn = np.zeros(m), np.zeros(m)
            done = 0
            for i in range(m):
                Z[i] = self.vcycle(V[i]) if precond else V[i]
                w = A @ Z[i]
                for l in range(i + 1):
                    H[l, i] = w @ V[l]
                    w -= H[l, i] * V[l]
                H[i + 1, i] = np.linalg.norm(w)
                if H[i + 1, i] > 0:
                    V[i + 1] = w / H[i + 1, i]
                for l in range(i):
                    t = cs[l] * H[l, i] + sn[l] * H[l + 1, i]
                    H[l + 1, i] = -sn[l] * H[l, i] + cs[l] * H[l + 1, i]
                    H[l, i] = t
                den = np.hypot(H[i, i], H[i + 1, i])
                cs[i], sn[i] = H[i, i] / den, H[i + 1, i] / den
                H[i, i] = den
                H[i + 1, i] = 0.0
                g[i + 1] = -sn[i] * g[i]
                g[i] = cs[i] * g[i]
                its += 1
                done = i + 1
                if abs(g[i + 1]) <= rtol * bn:
                    break
            y = np.linalg.solve(np.triu(H[:done, :done]), g[:done])
            x += Z[:done].T @ y
            if abs(g[done]) <= rtol * bn:
                break
        true = np.linalg.norm(b - A @ x) / bn
        return x, its, true


def evaluate(lev: Level, x, pts):
    """Velocity (n, 3) and pressure (n,) of the discrete function x at physical points."""
    S, rb, N = lev.sp, lev.rb, lev.N
    pts = np.atleast_2d(pts)
    cidx = np.minimum((pts * N).astype(int), N - 1)
    nu = len(rb.lu)
    U = np.zeros((len(pts), 3))
    Pv = np.zeros(len(pts))
    for n, (p, cc) in enumerate(zip(pts, cidx)):
        xi = (p * N - cc)[None, :]
        v, _ = rb.vel(xi)
        pv = rb.pres(xi)
        dofs = S.cell_dofs(tuple(cc))
        U[n] = np.einsum("i,ia->a", x[dofs[:nu]], v[:, 0, :])
        Pv[n] = x[dofs[nu:]] @ pv[:, 0]
    return U, Pv
