"""Quadrature assembly of the SIP-DG Stokes system (oracle; test
infrastructure only).

Everything here is evaluated literally from the paper's bilinear forms at
Gauss-Legendre points (k+2 per direction, exact for the polynomial
integrands): strain tensors, averages and jumps are built as 2x2 tensors and
contracted with ':'.  The GPU library uses closed modal formulas instead; the
two share no code.

Forms (Section 4):
  A_h  eq. (stiffness_form): volume 2 eta eps(u):eps(v); interior faces
       -{2 eta eps(u)}:[[v (x) n]] - {2 eta eps(v)}:[[u (x) n]]
       + sigma_F [[u (x) n]]:[[v (x) n]]; Navier faces
       -(n.2 eta eps(u) n)(v.n) - (n.2 eta eps(v) n)(u.n)
       + sigma_F (u.n)(v.n).
  eta_F                 eq. (eta_face): max of the two neighbours, eta_K on
                        the boundary.
  C_F, C_K              eq. (const_trace_face) and the discrete trace
                        lemma: C_K = (k+1)^2 |e| / |K|, C_F the max.
  gamma_F               eq. (sipg_penalty) at its lower bound with tau = 0
                        (Section 4.1 text after the coercivity proof):
                        4 eta_F on interior faces, 8 eta_F on Navier faces.
  sigma_F = gamma_F C_F (the face-wise penalty of Section 4).
  B_h  eq. (divergence_form): -div(u) q; {q}[[u.n]] on interior faces;
       q (u.n) on Navier faces.
  F, G eq. (rhs_f).
  S*   Section 5: pressure mass matrix scaled by 1/eta_K (diagonal in the
       orthonormal basis).

Reading for Dirichlet sides (not in the paper; used only for a manufactured
solution): the standard symmetric Nitsche/SIP boundary terms
  -(2 eta eps(u) n).v - (2 eta eps(v) n).u + sigma_F u.v
with the boundary penalty of a Navier face, the lift
  F += -(2 eta eps(v) n).g + sigma_F g.v,   G(q) = int q (g.n),
and B_h gets q (u.n) on Dirichlet faces as on Navier faces.

Basis: psi_ij(x, y) = (2/sqrt(h_x h_y)) lhat_i(xi) lhat_j(eta) with
lhat_i = sqrt((2i+1)/2) L_i, hence L2(K)-orthonormal (Section 5 states the
Legendre basis is pairwise orthogonal and the pressure basis orthonormal).

Precision: every assembly routine takes `dtype` (float64 by default).  With
numpy.longdouble the quadrature points, basis values, element sizes and all
products are carried in the 64-bit-mantissa type, which gives the matrices
to about 1e-19 relative: the reference against which residuals below the
FP64 rounding floor are measured (the extended-precision residual of
Section 8.3.1).
"""
import numpy as np
import scipy.sparse as sp

from .legendre import gauss, onb_derivs, onb_values
from .mesh import BOTTOM, DIRICHLET, LEFT, NAVIER, NEUMANN, RIGHT, TOP, Mesh

PENALTY_NF = 4.0  # n_F = number of faces of a quadrilateral, eq. (sipg_penalty)


# ----------------------------------------------------------------------------
# basis evaluation
# ----------------------------------------------------------------------------
def _h(mesh, dtype):
    """Element sizes l/n in the working type."""
    return (np.asarray(mesh.lx, dtype=dtype) / mesh.nx,
            np.asarray(mesh.ly, dtype=dtype) / mesh.ny)


def velocity_basis(k, hx, hy, xi, eta):
    """Vector basis phi_a, a = (d*(k+1) + j)*(k+1) + i, at reference points.

    Returns val[a, q, c] (component c of phi_a) and grad[a, q, c, r]
    (d/dx_r of component c)."""
    k1 = k + 1
    dt = np.asarray(xi).dtype
    c = 2 / np.sqrt(hx * hy)
    lx, dlx = onb_values(k, xi), onb_derivs(k, xi)
    ly, dly = onb_values(k, eta), onb_derivs(k, eta)
    nq = len(xi)
    nb = 2 * k1 * k1
    val = np.zeros((nb, nq, 2), dtype=dt)
    grad = np.zeros((nb, nq, 2, 2), dtype=dt)
    for d in range(2):
        for j in range(k1):
            for i in range(k1):
                a = (d * k1 + j) * k1 + i
                val[a, :, d] = c * lx[i] * ly[j]
                grad[a, :, d, 0] = c * (2 / hx) * dlx[i] * ly[j]
                grad[a, :, d, 1] = c * (2 / hy) * lx[i] * dly[j]
    return val, grad


def pressure_basis(k, hx, hy, xi, eta):
    """Scalar basis chi_m, m = j*k + i (0 <= i, j < k), values [m, q]."""
    dt = np.asarray(xi).dtype
    c = 2 / np.sqrt(hx * hy)
    if k < 1:
        return np.zeros((0, len(xi)), dtype=dt)
    lx, ly = onb_values(k - 1, xi), onb_values(k - 1, eta)
    out = np.zeros((k * k, len(xi)), dtype=dt)
    for j in range(k):
        for i in range(k):
            out[j * k + i] = c * lx[i] * ly[j]
    return out


def strain(grad):
    """eps(u) = (grad u + grad u^T)/2, acting on the last two axes."""
    return (grad + np.swapaxes(grad, -1, -2)) / 2


def _volume_points(k, dtype=np.float64):
    g, w = gauss(k + 2, dtype)
    xi, eta = np.meshgrid(g, g, indexing="xy")
    wq = np.outer(w, w)
    return xi.ravel(), eta.ravel(), wq.ravel()


def _side_points(k, side, hx, hy):
    """Reference points, physical line weights and outward normal on one side
    of an element (in the type of hx)."""
    dt = np.asarray(hx).dtype
    g, w = gauss(k + 2, dt)
    one = np.ones_like(g)
    if side == LEFT:
        return -one, g, w * hy / 2, np.array([-1, 0], dtype=dt)
    if side == RIGHT:
        return one, g, w * hy / 2, np.array([1, 0], dtype=dt)
    if side == BOTTOM:
        return g, -one, w * hx / 2, np.array([0, -1], dtype=dt)
    return g, one, w * hx / 2, np.array([0, 1], dtype=dt)


def trace_constant(k, side, hx, hy):
    """C_K = (k+1)^2 |e| / |K| (discrete trace lemma)."""
    e = hy if side in (LEFT, RIGHT) else hx
    return (k + 1) ** 2 * e / (hx * hy)


# ----------------------------------------------------------------------------
# reference (unit-coefficient) local matrices.  M[a, b] = form(u=phi_b, v=phi_a)
# ----------------------------------------------------------------------------
def volume_matrix(k, hx, hy):
    xi, eta, w = _volume_points(k, np.asarray(hx).dtype)
    w = w * hx * hy / 4
    _, grad = velocity_basis(k, hx, hy, xi, eta)
    eps = strain(grad)
    return 2 * np.einsum("aqcr,bqcr,q->ab", eps, eps, w)


def interior_face_unit_blocks(k, hx, hy, direction):
    """Unit blocks of the interior-face part of A_h.

    Side 0 is K^- (left for direction 0, below for direction 1), side 1 is
    K^+.  Returns T1, T2, T3 indexed [s][t] (trial side s, test side t):
      T1 multiplies eta_s   (from -{2 eta eps(u)}:[[v (x) n]])
      T2 multiplies eta_t   (from -{2 eta eps(v)}:[[u (x) n]])
      T3 multiplies sigma_F (from sigma_F [[u (x) n]]:[[v (x) n]])."""
    if direction == 0:
        sides = (RIGHT, LEFT)
    else:
        sides = (TOP, BOTTOM)
    pts = [_side_points(k, s, hx, hy) for s in sides]
    vals, epss, normals = [], [], []
    w = pts[0][2]
    for xi, eta, _, n in pts:
        v, gr = velocity_basis(k, hx, hy, xi, eta)
        vals.append(v)
        epss.append(strain(gr))
        normals.append(n)
    nb = vals[0].shape[0]
    T1 = [[None, None], [None, None]]
    T2 = [[None, None], [None, None]]
    T3 = [[None, None], [None, None]]
    for s in range(2):
        for t in range(2):
            # {2 eta eps(u)} with u on side s only = eta_s eps(u^s);
            # [[v (x) n]] with v on side t only = v^t (x) n^t.
            vt_n = np.einsum("aqc,r->aqcr", vals[t], normals[t])
            us_n = np.einsum("bqc,r->bqcr", vals[s], normals[s])
            T1[s][t] = -np.einsum("bqcr,aqcr,q->ab", epss[s], vt_n, w)
            T2[s][t] = -np.einsum("aqcr,bqcr,q->ab", epss[t], us_n, w)
            T3[s][t] = np.einsum("bqcr,aqcr,q->ab", us_n, vt_n, w)
            assert T1[s][t].shape == (nb, nb)
    return T1, T2, T3


def boundary_unit_blocks(k, hx, hy, side, kind):
    """Unit blocks (coefficient eta_K, eta_K, sigma_F) of one boundary side."""
    xi, eta, w, n = _side_points(k, side, hx, hy)
    val, grad = velocity_basis(k, hx, hy, xi, eta)
    eps2 = 2 * strain(grad)  # 2 eps(phi)
    if kind == NAVIER:
        nsn = np.einsum("c,aqcr,r->aq", n, eps2, n)  # n . 2 eps(phi) n
        vn = np.einsum("aqc,c->aq", val, n)  # phi . n
        B1 = -np.einsum("bq,aq,q->ab", nsn, vn, w)
        B2 = -np.einsum("aq,bq,q->ab", nsn, vn, w)
        B3 = np.einsum("bq,aq,q->ab", vn, vn, w)
    elif kind == DIRICHLET:
        sn = np.einsum("aqcr,r->aqc", eps2, n)  # 2 eps(phi) n
        B1 = -np.einsum("bqc,aqc,q->ab", sn, val, w)
        B2 = -np.einsum("aqc,bqc,q->ab", sn, val, w)
        B3 = np.einsum("bqc,aqc,q->ab", val, val, w)
    else:
        nb = val.shape[0]
        B1 = B2 = B3 = np.zeros((nb, nb), dtype=val.dtype)
    return B1, B2, B3


# ----------------------------------------------------------------------------
# face coefficients
# ----------------------------------------------------------------------------
def face_data(mesh: Mesh, eta, penalty_nf=PENALTY_NF, eta_override=None, dtype=np.float64):
    """Interior faces as arrays (minus, plus, eta_F, sigma_F) per direction and
    boundary faces as (side, element, eta_F, sigma_F).

    eta_override (optional scalar) replaces eta_F in the penalty by a global
    value (used only to contrast local and global penalties)."""
    k = mesh.k
    hx, hy = _h(mesh, dtype)
    eta = np.asarray(eta, dtype=dtype)
    out = {}
    faces = mesh.interior_faces()
    for direction in (0, 1):
        f = [(m, p) for m, p, dr in faces if dr == direction]
        m = np.array([a for a, _ in f], dtype=np.int64)
        p = np.array([b for _, b in f], dtype=np.int64)
        etaf = np.maximum(eta[m], eta[p]) if len(f) else np.zeros(0, dtype=dtype)
        side_m = RIGHT if direction == 0 else TOP
        side_p = LEFT if direction == 0 else BOTTOM
        cf = max(trace_constant(k, side_m, hx, hy),
                 trace_constant(k, side_p, hx, hy))
        etap = etaf if eta_override is None else np.full_like(etaf, eta_override)
        sigma = penalty_nf * etap * cf
        out[direction] = (m, p, etaf, sigma)
    bnd = []
    for side, e, fi in mesh.boundary_faces():
        kind = mesh.bc[side]
        etaf = eta[e]
        etap = etaf if eta_override is None else eta_override
        cf = trace_constant(k, side, hx, hy)
        sigma = penalty_nf * etap * 2 * cf if kind != NEUMANN else 0 * cf
        bnd.append((side, e, fi, kind, etaf, sigma))
    out["boundary"] = bnd
    return out


# ----------------------------------------------------------------------------
# global assembly
# ----------------------------------------------------------------------------
def _bsr(blocks_rows, blocks_cols, blocks, nrow_blocks, ncol_blocks):
    rows = np.asarray(blocks_rows, dtype=np.int64)
    cols = np.asarray(blocks_cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, data = rows[order], cols[order], blocks[order]
    indptr = np.zeros(nrow_blocks + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    br, bc = data.shape[1], data.shape[2]
    return sp.bsr_matrix((data, cols, indptr),
                         shape=(nrow_blocks * br, ncol_blocks * bc))


def assemble_A_blocks(mesh: Mesh, eta, penalty_nf=PENALTY_NF,
                      eta_override=None, dtype=np.float64):
    """Diagonal blocks (nel, nb, nb) and off-diagonal (row, col, block) lists
    of the SIP matrix A."""
    k = mesh.k
    hx, hy = _h(mesh, dtype)
    eta = np.asarray(eta, dtype=dtype)
    V = volume_matrix(k, hx, hy)
    diag = eta[:, None, None] * V[None]
    fd = face_data(mesh, eta, penalty_nf, eta_override, dtype)
    orow, ocol, oblk = [], [], []
    for direction in (0, 1):
        m, p, _, sigma = fd[direction]
        if len(m) == 0:
            continue
        T1, T2, T3 = interior_face_unit_blocks(k, hx, hy, direction)
        em, ep = eta[m], eta[p]
        s_ = sigma[:, None, None]
        # self blocks
        np.add.at(diag, m, em[:, None, None] * (T1[0][0] + T2[0][0])[None]
                  + s_ * T3[0][0][None])
        np.add.at(diag, p, ep[:, None, None] * (T1[1][1] + T2[1][1])[None]
                  + s_ * T3[1][1][None])
        # coupling: row = test element, col = trial element
        blk_mp = (ep[:, None, None] * T1[1][0][None]
                  + em[:, None, None] * T2[1][0][None] + s_ * T3[1][0][None])
        blk_pm = (em[:, None, None] * T1[0][1][None]
                  + ep[:, None, None] * T2[0][1][None] + s_ * T3[0][1][None])
        orow += [m, p]
        ocol += [p, m]
        oblk += [blk_mp, blk_pm]
    cache = {}
    for side, e, fi, kind, etaf, sigma in fd["boundary"]:
        if kind == NEUMANN:
            continue
        key = (side, kind)
        if key not in cache:
            cache[key] = boundary_unit_blocks(k, hx, hy, side, kind)
        B1, B2, B3 = cache[key]
        diag[e] += eta[e] * (B1 + B2) + sigma * B3
    if orow:
        orow = np.concatenate(orow)
        ocol = np.concatenate(ocol)
        oblk = np.concatenate(oblk)
    else:
        nb = mesh.nbu
        orow = ocol = np.zeros(0, dtype=np.int64)
        oblk = np.zeros((0, nb, nb), dtype=dtype)
    return diag, (orow, ocol, oblk)


def assemble_A(mesh: Mesh, eta, penalty_nf=PENALTY_NF, eta_override=None,
               dtype=np.float64):
    """Sparse (BSR) SIP matrix A, A[a, b] = A_h(phi_b, phi_a)."""
    diag, (orow, ocol, oblk) = assemble_A_blocks(mesh, eta, penalty_nf,
                                                 eta_override, dtype)
    nel = mesh.nel
    rows = np.concatenate([np.arange(nel), orow])
    cols = np.concatenate([np.arange(nel), ocol])
    blocks = np.concatenate([diag, oblk])
    return _bsr(rows, cols, blocks, nel, nel)


def assemble_B(mesh: Mesh, dtype=np.float64):
    """Sparse B, B[a, m] = B_h(phi_a, chi_m) (velocity rows, pressure cols)."""
    k = mesh.k
    hx, hy = _h(mesh, dtype)
    nel = mesh.nel
    xi, et, w = _volume_points(k, dtype)
    w = w * hx * hy / 4
    _, grad = velocity_basis(k, hx, hy, xi, et)
    chi = pressure_basis(k, hx, hy, xi, et)
    div = grad[:, :, 0, 0] + grad[:, :, 1, 1]
    Bvol = -np.einsum("aq,mq,q->am", div, chi, w)
    rows = [np.arange(nel)]
    cols = [np.arange(nel)]
    blks = [np.repeat(Bvol[None], nel, axis=0)]
    for direction in (0, 1):
        faces = [(m, p) for m, p, dr in mesh.interior_faces() if dr == direction]
        if not faces:
            continue
        sides = (RIGHT, LEFT) if direction == 0 else (TOP, BOTTOM)
        vn, ch = [], []
        for s in sides:
            xs, ys, wf, n = _side_points(k, s, hx, hy)
            v, _ = velocity_basis(k, hx, hy, xs, ys)
            vn.append(np.einsum("aqc,c->aq", v, n))
            ch.append(pressure_basis(k, hx, hy, xs, ys))
        m = np.array([a for a, _ in faces])
        p = np.array([b for _, b in faces])
        el = (m, p)
        # {q}[[v.n]] with q on side s, v on side t: 1/2 q^s (v^t . n^t)
        for s in range(2):
            for t in range(2):
                blk = np.einsum("aq,mq,q->am", vn[t], ch[s], wf) / 2
                rows.append(el[t])
                cols.append(el[s])
                blks.append(np.repeat(blk[None], len(m), axis=0))
    for side, e, fi in mesh.boundary_faces():
        if mesh.bc[side] == NEUMANN:
            continue
        xs, ys, wf, n = _side_points(k, side, hx, hy)
        v, _ = velocity_basis(k, hx, hy, xs, ys)
        ch = pressure_basis(k, hx, hy, xs, ys)
        blk = np.einsum("aqc,c,mq,q->am", v, n, ch, wf)
        rows.append(np.array([e]))
        cols.append(np.array([e]))
        blks.append(blk[None])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    blks = np.concatenate(blks)
    # sum duplicate (row, col) blocks before building the BSR structure
    key = rows * nel + cols
    uk, inv = np.unique(key, return_inverse=True)
    summed = np.zeros((len(uk),) + blks.shape[1:], dtype=dtype)
    np.add.at(summed, inv, blks)
    return _bsr(uk // nel, uk % nel, summed, nel, nel)


def face_basis(k, length, tau):
    """Face-orthonormal basis sqrt(2/|e|) lhat_m(tau), shape (k+1, nq)."""
    return np.sqrt(2 / length) * onb_values(k, tau)


def assemble_rhs(mesh: Mesh, eta, f, g=None, penalty_nf=PENALTY_NF, dtype=np.float64):
    """F (velocity) and G (pressure) right-hand sides.

    f: modal body force, shape (nel, 2, k+1, k+1); F = int f.v = f because the
    basis is orthonormal.  g: Dirichlet data (nbfaces, 2, k+1) or None."""
    k = mesh.k
    hx, hy = _h(mesh, dtype)
    F = np.array(f, dtype=dtype).reshape(-1).copy()
    G = np.zeros(mesh.np_, dtype=dtype)
    if g is None or all(b != DIRICHLET for b in mesh.bc):
        return F, G
    g = np.asarray(g, dtype=dtype).reshape(mesh.nbfaces(), 2, k + 1)
    eta = np.asarray(eta, dtype=dtype)
    fd = face_data(mesh, eta, penalty_nf, dtype=dtype)
    nbu, nbp = mesh.nbu, mesh.nbp
    for side, e, fi, kind, etaf, sigma in fd["boundary"]:
        if kind != DIRICHLET:
            continue
        xs, ys, wf, n = _side_points(k, side, hx, hy)
        tau = ys if side in (LEFT, RIGHT) else xs
        length = hy if side in (LEFT, RIGHT) else hx
        gq = np.einsum("dm,mq->qd", g[fi], face_basis(k, length, tau))
        val, grad = velocity_basis(k, hx, hy, xs, ys)
        sn = np.einsum("aqcr,r->aqc", 2 * strain(grad), n)
        lift = (-eta[e] * np.einsum("aqc,qc,q->a", sn, gq, wf)
                + sigma * np.einsum("aqc,qc,q->a", val, gq, wf))
        F[e * nbu:(e + 1) * nbu] += lift
        ch = pressure_basis(k, hx, hy, xs, ys)
        G[e * nbp:(e + 1) * nbp] += np.einsum("mq,qc,c,q->m", ch, gq, n, wf)
    return F, G


def schur_diag(mesh: Mesh, eta):
    """Diagonal of S* (Section 5): pressure mass / eta_K, orthonormal basis."""
    return np.repeat(1.0 / np.asarray(eta, dtype=np.float64), mesh.nbp)


def pressure_mean_vector(mesh: Mesh):
    """c with c.p = int_Omega p: only the constant mode, int psi_00 = sqrt|K|."""
    c = np.zeros(mesh.np_)
    c[::mesh.nbp] = np.sqrt(mesh.hx * mesh.hy)
    return c


# ----------------------------------------------------------------------------
# element-block Jacobi form, eq. (smoother), evaluated directly
# ----------------------------------------------------------------------------
def smoother_blocks_from_form(mesh: Mesh, eta, penalty_nf=PENALTY_NF):
    """Per-element matrices of the block-Jacobi bilinear form of eq.
    (smoother): the volume term, on each interior face of K the one-sided
    terms -eta^K eps(u^K):(v^K (x) n^K) - eta^K eps(v^K):(u^K (x) n^K)
    + sigma_F (u^K (x) n^K):(v^K (x) n^K), plus the boundary terms.  Written
    independently of the global assembly, to check that it equals the
    diagonal blocks of A."""
    k, hx, hy = mesh.k, mesh.hx, mesh.hy
    eta = np.asarray(eta, dtype=np.float64)
    V = volume_matrix(k, hx, hy)
    fd = face_data(mesh, eta, penalty_nf)
    sig = {}
    for direction in (0, 1):
        m, p, _, s = fd[direction]
        for a, b, sv in zip(m, p, s):
            if direction == 0:
                sig[(a, RIGHT)] = sv
                sig[(b, LEFT)] = sv
            else:
                sig[(a, TOP)] = sv
                sig[(b, BOTTOM)] = sv
    bsig = {(e, side): (kind, sv)
            for side, e, fi, kind, _, sv in fd["boundary"]}
    one_sided = {}
    for side in (LEFT, RIGHT, BOTTOM, TOP):
        xs, ys, wf, n = _side_points(k, side, hx, hy)
        val, grad = velocity_basis(k, hx, hy, xs, ys)
        eps = strain(grad)
        v_n = np.einsum("aqc,r->aqcr", val, n)
        c1 = -np.einsum("bqcr,aqcr,q->ab", eps, v_n, wf)
        c2 = -np.einsum("aqcr,bqcr,q->ab", eps, v_n, wf)
        c3 = np.einsum("bqcr,aqcr,q->ab", v_n, v_n, wf)
        one_sided[side] = (c1, c2, c3)
    out = np.zeros((mesh.nel, mesh.nbu, mesh.nbu))
    for e in range(mesh.nel):
        M = eta[e] * V
        for side in (LEFT, RIGHT, BOTTOM, TOP):
            if (e, side) in sig:
                c1, c2, c3 = one_sided[side]
                M = M + eta[e] * (c1 + c2) + sig[(e, side)] * c3
            else:
                kind, sv = bsig[(e, side)]
                if kind != NEUMANN:
                    B1, B2, B3 = boundary_unit_blocks(k, hx, hy, side, kind)
                    M = M + eta[e] * (B1 + B2) + sv * B3
        out[e] = M
    return out
