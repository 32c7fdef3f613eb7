"""Exact references for the lattice N-body Coulomb energy (test infrastructure).

TEST INFRASTRUCTURE ONLY; never imported by the product path.

The heat-bath chain samples the Gaussian law e^{-H_L} with
H_L = 1/2 sum_<m,n> (phi_m - phi_n)^2 (the paper's lattice action, Eq.
proplat), Dirichlet ghosts phi = 0 outside the box.  Its covariance is the
lattice Green's function G = (-Delta_L)^{-1} with -Delta_L = 6 I - adjacency
on the box.  The field average of Eq. (nsum) is therefore exactly

    E_lat = sum_{i != j} q_i q_j G(n_i, n_j) = q^T G q - sum_i q_i^2 G(n_i, n_i),

which the Monte-Carlo mean (Eq. nsum2) estimates without bias.  This module
computes E_lat by several independent routes, plus the continuum sum of the
paper's Eq. (s1) and the infinite-lattice Green's function whose large-r
limit is 1/(4 pi r) (Eq. path and Eq. proplat).

Routes:
  * dense Cholesky of -Delta_L (small boxes, e.g. 16^3 -> 4096 x 4096);
  * DST-I spectral solve: -Delta_L is a Kronecker sum of 1-D Dirichlet
    Laplacians tridiag(-1, 2, -1), diagonalised by the type-I sine transform
    with eigenvalues 2 - 2 cos(pi k / (L + 1)), k = 1..L (any box size);
  * conjugate gradients on the sparse -Delta_L (cross-check);
  * G(n, n) from the heat kernel, G = int_0^inf exp(-t (-Delta_L)) dt, whose
    diagonal factorises over the three axes;
  * off-lattice charges (spread over the 8 corners of their cell with
    trilinear weights w_i): the interpolated field phi~(r_i) = w_i^T phi has
    covariance w_i^T G w_j, so the estimator's mean is
    E = sum_{i != j} q_i q_j w_i^T G w_j = rho^T G rho - sum_i q_i^2 w_i^T G w_i
    with rho = sum_i q_i w_i, and dE/dr_i = 2 q_i (dw_i/dr_i)^T G (rho - q_i w_i);
  * infinite lattice: G_inf(n) = int_0^inf e^{-6t} I_nx(2t) I_ny(2t) I_nz(2t) dt;
    G_inf(0) equals Watson's simple-cubic integral divided by 6, which has
    the closed form sqrt(6)/(32 pi^3) Gamma(1/24) Gamma(5/24) Gamma(7/24)
    Gamma(11/24) (Glasser and Zucker, 1977).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.integrate
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg
import scipy.special

__all__ = [
    "laplacian_dense", "laplacian_sparse", "green_dense", "energy_dense",
    "qGq_dst", "green_diag_heat", "green_diag_modes", "energy_dst", "solve_cg",
    "green_infinite", "watson_closed_form", "energy_continuum", "gaussian_var_O",
    "cic_corners", "energy_offlattice_dense", "grad_offlattice_dense",
]


def _lin(shape, xyz):
    lx, ly, _ = shape
    xyz = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    return xyz[:, 0] + lx * (xyz[:, 1] + ly * xyz[:, 2])


def laplacian_sparse(shape) -> scipy.sparse.csr_matrix:
    """-Delta_L = 6 I - adjacency on the box, Dirichlet ghosts (CSR, FP64).
    Linear index x + lx*(y + ly*z)."""
    lx, ly, lz = shape

    def lap1(n):
        return scipy.sparse.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])

    ix, iy, iz = (scipy.sparse.identity(n) for n in (lx, ly, lz))
    # Kronecker sum; x is the fastest index, so it is the last Kronecker factor
    A = (scipy.sparse.kron(scipy.sparse.kron(iz, iy), lap1(lx))
         + scipy.sparse.kron(scipy.sparse.kron(iz, lap1(ly)), ix)
         + scipy.sparse.kron(scipy.sparse.kron(lap1(lz), iy), ix))
    return A.tocsr()


def laplacian_dense(shape) -> np.ndarray:
    """Dense -Delta_L built site by site from the nearest-neighbour pairs."""
    lx, ly, lz = shape
    V = lx * ly * lz
    A = np.zeros((V, V))
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                i = x + lx * (y + ly * z)
                A[i, i] = 6.0
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    a, b, c = x + dx, y + dy, z + dz
                    if 0 <= a < lx and 0 <= b < ly and 0 <= c < lz:
                        A[i, a + lx * (b + ly * c)] = -1.0
    return A


def green_dense(shape) -> np.ndarray:
    """Full G = (-Delta_L)^{-1} by Cholesky (small boxes only)."""
    A = laplacian_dense(shape)
    cf = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(cf, np.eye(A.shape[0]))


def energy_dense(shape, xyz, q, G: np.ndarray | None = None) -> float:
    """E_lat = sum_{i != j} q_i q_j G(n_i, n_j), summed pair by pair from
    the Cholesky Green's function (co-located charges i != j included)."""
    if G is None:
        G = green_dense(shape)
    s = _lin(shape, xyz)
    q = np.asarray(q, dtype=np.float64)
    Gs = G[np.ix_(s, s)]
    M = np.outer(q, q) * Gs
    np.fill_diagonal(M, 0.0)
    return float(M.sum())


def _dst_eigen(shape):
    lams = [2.0 - 2.0 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1)) for n in shape]
    lx, ly, lz = shape
    # array order (z, y, x)
    return (lams[2][:, None, None] + lams[1][None, :, None] + lams[0][None, None, :])


def qGq_dst(shape, xyz, q) -> float:
    """q^T G q = sum_k |rho_hat_k|^2 / lambda_k with rho the charge grid and
    rho_hat its orthonormal DST-I (exact for the Dirichlet box)."""
    lx, ly, lz = shape
    rho = np.zeros((lz, ly, lx))
    xyz = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    np.add.at(rho, (xyz[:, 2], xyz[:, 1], xyz[:, 0]), np.asarray(q, dtype=np.float64))
    rh = scipy.fft.dstn(rho, type=1, norm="ortho", workers=-1)
    return float(np.sum(rh * rh / _dst_eigen(shape)))


def _heat_1d_diag(n: int, t: np.ndarray) -> np.ndarray:
    """[exp(-t A_1)]_{xx} for the 1-D Dirichlet Laplacian A_1 of size n:
    sum_k 2/(n+1) sin^2(pi k (x+1)/(n+1)) exp(-t lambda_k); shape (n, len(t))."""
    k = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    x = np.arange(n)
    v2 = (2.0 / (n + 1)) * np.sin(np.pi * np.outer(x + 1, k) / (n + 1)) ** 2  # (n, k)
    return v2 @ np.exp(-np.outer(lam, t))


def green_diag_heat(shape, xyz, h: float = 0.04) -> np.ndarray:
    """G(n, n) = int_0^inf prod_mu [exp(-t A_mu)]_{n_mu n_mu} dt, trapezoid
    rule in u = log t (integrand e^u prod(...), smooth and decaying at both
    ends)."""
    lx, ly, lz = shape
    lam_min = sum(2.0 - 2.0 * np.cos(np.pi / (n + 1)) for n in shape)
    u_hi = math.log(60.0 / lam_min)
    u = np.arange(-36.0, u_hi + h, h)
    t = np.exp(u)
    Kx, Ky, Kz = (_heat_1d_diag(n, t) for n in (lx, ly, lz))
    xyz = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    out = np.empty(xyz.shape[0])
    w = t * h
    for a in range(0, xyz.shape[0], 8192):
        b = slice(a, a + 8192)
        out[b] = (Kx[xyz[b, 0]] * Ky[xyz[b, 1]] * Kz[xyz[b, 2]]) @ w
    return out


def green_diag_modes(shape, xyz) -> np.ndarray:
    """G(n, n) = sum over all DST-I modes of prod_mu v_k(n_mu)^2 / lambda_k
    (direct mode sum, O(V) per site; small boxes)."""
    lx, ly, lz = shape
    lam = _dst_eigen(shape)
    out = []
    for x, y, z in np.asarray(xyz, dtype=np.int64).reshape(-1, 3):
        vs = []
        for n, c in ((lx, x), (ly, y), (lz, z)):
            k = np.arange(1, n + 1)
            vs.append((2.0 / (n + 1)) * np.sin(np.pi * k * (c + 1) / (n + 1)) ** 2)
        out.append(float(np.sum(vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :] / lam)))
    return np.array(out)


def energy_dst(shape, xyz, q) -> float:
    """E_lat = q^T G q - sum_i q_i^2 G(n_i, n_i) with q^T G q from the DST-I
    solve and the diagonal from the heat kernel (any box size)."""
    q = np.asarray(q, dtype=np.float64)
    return qGq_dst(shape, xyz, q) - float(np.sum(q * q * green_diag_heat(shape, xyz)))


def solve_cg(shape, rhs: np.ndarray, rtol: float = 1e-13) -> np.ndarray:
    """u = G rhs by conjugate gradients on the sparse -Delta_L (FP64)."""
    A = laplacian_sparse(shape)
    u, info = scipy.sparse.linalg.cg(A, rhs, rtol=rtol, atol=0.0, maxiter=100000)
    if info != 0:
        raise RuntimeError(f"CG did not converge (info={info})")
    return u


def green_infinite(n) -> float:
    """Infinite-lattice Green's function of 6 I - adjacency at offset n:
    int_0^inf e^{-6t} I_nx(2t) I_ny(2t) I_nz(2t) dt (modified Bessel I, via
    the exponentially scaled ive so the integrand is prod ive(n_mu, 2t))."""
    nx, ny, nz = (abs(int(v)) for v in n)

    def f(t):
        return (scipy.special.ive(nx, 2 * t) * scipy.special.ive(ny, 2 * t)
                * scipy.special.ive(nz, 2 * t))

    # integrand ~ (4 pi t)^{-3/2} for large t: integrate to T numerically and
    # add the tail of the leading asymptote plus its first correction.
    T = 4.0e4
    pieces = [0.0, 1.0, 10.0, 100.0, 1000.0, 1.0e4, T]
    s = 0.0
    for a, b in zip(pieces[:-1], pieces[1:]):
        s += scipy.integrate.quad(f, a, b, limit=400, epsabs=0.0, epsrel=1e-13)[0]
    # large-t expansion: ive(n, 2t) ~ e^{0}/sqrt(4 pi t) (1 - (4n^2-1)/(16 t) + ...)
    c = sum((4 * m * m - 1) / 16.0 for m in (nx, ny, nz))
    a0 = (4 * math.pi) ** -1.5
    tail = a0 * (2.0 / math.sqrt(T) - c * (2.0 / 3.0) * T ** -1.5)
    return s + tail


def watson_closed_form() -> float:
    """G_inf(0) = W / 6 with Watson's simple-cubic integral
    W = sqrt(6)/(32 pi^3) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)."""
    g = math.gamma
    W = math.sqrt(6.0) / (32.0 * math.pi ** 3) * g(1 / 24) * g(5 / 24) * g(7 / 24) * g(11 / 24)
    return W / 6.0


def energy_continuum(xyz, q) -> float:
    """The paper's Eq. (s1): (1/(4 pi)) sum over ordered pairs i != j of
    q_i q_j / |r_i - r_j| (lattice spacing 1; sites must be distinct)."""
    r = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    s = 0.0
    for i in range(r.shape[0]):
        d = np.sqrt(np.sum((r - r[i]) ** 2, axis=1))
        d[i] = np.inf
        s += float(np.sum(q[i] * q / d))
    return s / (4.0 * math.pi)


def gaussian_var_O(Gss: np.ndarray, q: np.ndarray) -> float:
    """Var(O) for O = X^2 - Y, X = sum q_i phi_i, Y = sum q_i^2 phi_i^2 when
    phi is Gaussian with covariance G restricted to the charge sites (Gss),
    by Wick's theorem: Var(X^2) = 2 (q^T G q)^2, Var(Y) = 2 sum_ij q_i^2 q_j^2
    G_ij^2, Cov(X^2, Y) = 2 sum_j q_j^2 ((G q)_j)^2."""
    q = np.asarray(q, dtype=np.float64)
    s = float(q @ Gss @ q)
    Gq = Gss @ q
    q2 = q * q
    var_x2 = 2.0 * s * s
    var_y = 2.0 * float(q2 @ (Gss * Gss) @ q2)
    cov = 2.0 * float(np.sum(q2 * Gq * Gq))
    return var_x2 + var_y - 2.0 * cov


def cic_corners(shape, r):
    """For charges at real positions r (n x 3, lattice units, site (x,y,z) at
    (x,y,z), 0 <= r_d <= L_d - 1): the natural linear indices of the 8
    corners of each charge's cell (origin min(floor(r_d), L_d - 2)), their
    trilinear weights, and the weights' derivatives with respect to r
    (n x 8 x 3)."""
    L = np.asarray(shape, dtype=np.int64)
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    b = np.minimum(np.floor(r), (L - 2)[None, :]).astype(np.int64)
    f = r - b
    e = np.array([[ex, ey, ez] for ez in (0, 1) for ey in (0, 1) for ex in (0, 1)])  # 8 x 3
    corner = b[:, None, :] + e[None, :, :]  # n x 8 x 3
    idx = corner[..., 0] + L[0] * (corner[..., 1] + L[1] * corner[..., 2])
    fac = np.where(e[None, :, :] == 1, f[:, None, :], 1.0 - f[:, None, :])  # n x 8 x 3 per-axis factors
    w = fac.prod(axis=2)
    sign = np.where(e == 1, 1.0, -1.0)  # d(factor_d)/d r_d
    dw = np.empty(w.shape + (3,))
    for d in range(3):
        others = [k for k in range(3) if k != d]
        dw[..., d] = sign[None, :, d] * fac[..., others[0]] * fac[..., others[1]]
    return idx, w, dw


def _cic_matrices(shape, r, q):
    idx, w, dw = cic_corners(shape, r)
    V = int(np.prod(shape))
    n = idx.shape[0]
    W = np.zeros((n, V))
    np.add.at(W, (np.repeat(np.arange(n), 8), idx.ravel()), w.ravel())
    return idx, w, dw, W


def energy_offlattice_dense(shape, r, q, G: np.ndarray | None = None) -> float:
    """E = sum_{i != j} q_i q_j w_i^T G w_j for charges at real positions,
    from the Cholesky Green's function (small boxes)."""
    if G is None:
        G = green_dense(shape)
    q = np.asarray(q, dtype=np.float64)
    _, _, _, W = _cic_matrices(shape, r, q)
    C = W @ G @ W.T  # covariance of the interpolated field at the charges
    M = np.outer(q, q) * C
    np.fill_diagonal(M, 0.0)
    return float(M.sum())


def grad_offlattice_dense(shape, r, q, G: np.ndarray | None = None) -> np.ndarray:
    """dE/dr_i (n x 3) of the off-lattice energy above:
    2 q_i (dw_i/dr_i)^T G (rho - q_i w_i), rho = sum_j q_j w_j."""
    if G is None:
        G = green_dense(shape)
    q = np.asarray(q, dtype=np.float64)
    idx, w, dw, W = _cic_matrices(shape, r, q)
    rho = W.T @ q
    out = np.zeros((q.shape[0], 3))
    for i in range(q.shape[0]):
        u = G @ (rho - q[i] * W[i])
        out[i] = 2.0 * q[i] * (dw[i].T @ u[idx[i]])
    return out
