"""Random-feature-method collocation systems for -Laplace(u) = f (and the 3D
Helmholtz problem of Example 4.5) on the unit cube.

Discretisation (Sec. 2.1 of the paper, eqs. (2.1)-(2.3); hyper-parameters of
Appendix B): the domain [0,1]^d is split into N^d boxes with centre c_q and
radius r = 1/(2N).  Box q carries J features

    phi_qj(x) = tanh( w_qj . (x - c_q) / r + b_qj ),   w, b ~ U[-1, 1]  (R = 1)

and the PoU is the indicator psi^a, so continuity between boxes is imposed by
extra C0 / C1 rows.  Rows of A (all with unit penalty weights):

* interior:  -Laplace(phi) = 2 t (1 - t^2) |w|^2 / r^2          (t = tanh(.))
  at Q^d cell-centred points per box, right-hand side f;
* Dirichlet: phi at Q^(d-1) cell-centred points per boundary box face, rhs g = u;
* interface: per shared face, Q^(d-1) cell-centred points, each giving a C0 row
  (phi_p - phi_q) and a C1 row (d_n phi_p - d_n phi_q, d_k phi = (1-t^2) w_k / r),
  rhs 0.

Row order: interior (box-major, points row-major), Dirichlet (face by face:
axis 0 low/high, axis 1 low/high, ...; boxes ascending; points row-major),
interfaces (axis-major, lower box ascending, points row-major; C0 then C1).
Columns are box-major: column q*J + j.  Within a row the columns ascend (the
lower box of an interface always has the smaller index).

Manufactured solution u = sin(k pi x_0) prod_{i>0} sin(pi x_i), so
f = (k^2 + d - 1) pi^2 u.  k = 1 gives the single right-hand side; k = 1..32 the
batched one.

The same construction with pde="helmholtz" gives the three-dimensional
Helmholtz problem of Example 4.5: Laplace(u) + kappa^2 u = f with Dirichlet
data, kappa = 0.5 (the paper's wave number), interior rows
Laplace(phi) + kappa^2 phi = -2 t (1 - t^2) |w|^2 / r^2 + kappa^2 t, and the
paper's manufactured solution
    u = -a prod_i cos(pi x_i + 2 pi/5)
        -b cos(pi x + 2 pi/5) cos(2 pi y + 2 pi/5) cos(4 pi z + 2 pi/5),
mode 1 = low frequency (a, b) = (1, 0), mode 2 = high (0, 1), mode 3 = mixed
(0.5, 0.5); f = (kappa^2 - 3 pi^2) u_a + (kappa^2 - 21 pi^2) u_b.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class RFMSystem:
    d: int
    N: int
    J: int
    Q: int
    m: int
    n: int
    row_ptr: np.ndarray  # int64[m+1]
    col: np.ndarray  # int32[nnz], ascending within a row
    val: np.ndarray  # float64[nnz]
    b: np.ndarray  # float64[nrhs, m] (row k = right-hand side k, contiguous)
    modes: tuple
    centres: np.ndarray  # float64[N^d, d]
    radius: float
    W: np.ndarray  # float64[N^d, J, d]
    B0: np.ndarray  # float64[N^d, J]
    counts: dict = field(default_factory=dict)
    pde: str = "poisson"
    kwave: float = 0.0

    def exact(self, pts: np.ndarray, k: int = 1) -> np.ndarray:
        """The manufactured solution of right-hand side mode k at pts."""
        return exact_solution(pts, k, self.pde)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def nrhs(self) -> int:
        return self.b.shape[0]


# Workload definitions.  Sizes follow the problem statement of each workload:
#   poisson2d_2x2   : 2x2 boxes, J=50,  Q=20  -> m=1,920,   n=200,    s=4n
#   poisson2d_8x8   : 8x8 boxes, J=200, Q=40  -> m=112,640, n=12,800, s=4n
#   poisson3d_4x4x4 : 4^3 boxes, J=400, Q=12  -> m=165,888, n=25,600, s=2n
# plus small intermediate systems used by the parity tests.
CONFIGS = {
    "poisson2d_2x2": dict(d=2, N=2, J=50, Q=20, gamma=4),
    "poisson2d_8x8": dict(d=2, N=8, J=200, Q=40, gamma=4),
    "poisson3d_4x4x4": dict(d=3, N=4, J=400, Q=12, gamma=2),
    # intermediate sizes: several tiles and a ragged tail for the kernels
    "poisson2d_3x3": dict(d=2, N=3, J=70, Q=18, gamma=4),  # n=630
    "poisson2d_4x4": dict(d=2, N=4, J=100, Q=24, gamma=4),  # n=1,600
    "poisson3d_2x2x2": dict(d=3, N=2, J=90, Q=8, gamma=2),  # n=720
    # Example 4.5 (3D Helmholtz, kappa = 0.5) on the paper's 2x2x2 boxes with its
    # smallest feature count (J = 400 per box, 20 points per axis):
    #   m = 64,000 + 9,600 + 9,600 = 83,200, n = 3,200, s = 4n
    "helmholtz3d_2x2x2": dict(d=3, N=2, J=400, Q=20, gamma=4, pde="helmholtz", kwave=0.5),
    "helmholtz3d_2x2x2_small": dict(d=3, N=2, J=90, Q=8, gamma=2, pde="helmholtz", kwave=0.5),  # n=720
}

FEATURE_SEED = 1
SAMPLE_POINT_SEED = 3
CONSISTENT_RHS_SEED = 4


def _cell_centres(lo: np.ndarray, hi: np.ndarray, Q: int) -> np.ndarray:
    """Q points per axis, cell-centred in [lo, hi] for each axis; row-major."""
    axes = [lo[k] + (np.arange(Q) + 0.5) * (hi[k] - lo[k]) / Q for k in range(len(lo))]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def _box_index(ijk, N):
    idx = 0
    for c in ijk:
        idx = idx * N + c
    return idx


HELMHOLTZ_MODES = {1: (1.0, 0.0), 2: (0.0, 1.0), 3: (0.5, 0.5)}  # low, high, mixed (a, b)


def _helmholtz_parts(pts: np.ndarray):
    ph = 2.0 * np.pi / 5.0
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    ua = -np.cos(np.pi * x + ph) * np.cos(np.pi * y + ph) * np.cos(np.pi * z + ph)
    ub = -np.cos(np.pi * x + ph) * np.cos(2 * np.pi * y + ph) * np.cos(4 * np.pi * z + ph)
    return ua, ub


def exact_solution(pts: np.ndarray, k: int = 1, pde: str = "poisson") -> np.ndarray:
    if pde == "helmholtz":
        a, b = HELMHOLTZ_MODES[k]
        ua, ub = _helmholtz_parts(pts)
        return a * ua + b * ub
    u = np.sin(k * np.pi * pts[:, 0])
    for i in range(1, pts.shape[1]):
        u = u * np.sin(np.pi * pts[:, i])
    return u


def _rhs_f(pts: np.ndarray, k: int, pde: str = "poisson", kwave: float = 0.0) -> np.ndarray:
    if pde == "helmholtz":
        a, b = HELMHOLTZ_MODES[k]
        ua, ub = _helmholtz_parts(pts)
        # Laplace(u_a) = -3 pi^2 u_a, Laplace(u_b) = -(1 + 4 + 16) pi^2 u_b
        return a * (kwave ** 2 - 3 * np.pi ** 2) * ua + b * (kwave ** 2 - 21 * np.pi ** 2) * ub
    d = pts.shape[1]
    return (k * k + d - 1) * np.pi ** 2 * exact_solution(pts, k)


def _features(sys_c: np.ndarray, r: float, W: np.ndarray, B0: np.ndarray, pts: np.ndarray):
    """t = tanh(w.(x-c)/r + b) for all J features of one box at all pts -> (P, J)."""
    z = ((pts - sys_c) / r) @ W.T + B0
    return np.tanh(z)


def poisson_system(d: int, N: int, J: int, Q: int, modes=(1,), seed: int = FEATURE_SEED,
                   pde: str = "poisson", kwave: float = 0.0) -> RFMSystem:
    if pde not in ("poisson", "helmholtz") or (pde == "helmholtz" and d != 3):
        raise ValueError("pde is 'poisson' (d = 2, 3) or 'helmholtz' (d = 3)")
    nbox = N ** d
    r = 1.0 / (2 * N)
    boxes = list(itertools.product(range(N), repeat=d))
    centres = np.array([[(2 * a + 1) * r for a in bx] for bx in boxes], dtype=np.float64)
    rng = np.random.default_rng(seed)
    draws = rng.uniform(-1.0, 1.0, size=(nbox, J, d + 1))
    W = np.ascontiguousarray(draws[:, :, :d])
    B0 = np.ascontiguousarray(draws[:, :, d])
    n = nbox * J
    modes = tuple(int(k) for k in modes)

    blocks_cols, blocks_vals, rhs = [], [], []
    counts = {"interior": 0, "dirichlet": 0, "interface": 0}

    def add(cols: np.ndarray, vals: np.ndarray, b_rows: np.ndarray):
        blocks_cols.append(cols)
        blocks_vals.append(vals)
        rhs.append(b_rows)

    # interior rows
    for q, bx in enumerate(boxes):
        lo = centres[q] - r
        hi = centres[q] + r
        pts = _cell_centres(lo, hi, Q)
        t = _features(centres[q], r, W[q], B0[q], pts)
        wn2 = (W[q] ** 2).sum(axis=1) / (r * r)
        lap = 2.0 * t * (1.0 - t * t) * wn2[None, :]  # -Laplace(phi)
        vals = lap if pde == "poisson" else kwave ** 2 * t - lap
        cols = np.broadcast_to(q * J + np.arange(J, dtype=np.int64), vals.shape)
        add(cols, vals, np.stack([_rhs_f(pts, k, pde, kwave) for k in modes], axis=0))
        counts["interior"] += pts.shape[0]

    # Dirichlet rows
    for axis in range(d):
        for side in (0, 1):
            for q, bx in enumerate(boxes):
                if bx[axis] != (0 if side == 0 else N - 1):
                    continue
                lo = centres[q] - r
                hi = centres[q] + r
                other = [a for a in range(d) if a != axis]
                face = _cell_centres(lo[other], hi[other], Q)
                pts = np.empty((face.shape[0], d))
                pts[:, other] = face
                pts[:, axis] = float(side)
                t = _features(centres[q], r, W[q], B0[q], pts)
                cols = np.broadcast_to(q * J + np.arange(J, dtype=np.int64), t.shape)
                add(cols, t, np.stack([exact_solution(pts, k, pde) for k in modes], axis=0))
                counts["dirichlet"] += pts.shape[0]

    # interface rows (C0 then C1 per point)
    for axis in range(d):
        for p, bx in enumerate(boxes):
            if bx[axis] == N - 1:
                continue
            nb = list(bx)
            nb[axis] += 1
            qb = _box_index(nb, N)
            lo = centres[p] - r
            hi = centres[p] + r
            other = [a for a in range(d) if a != axis]
            face = _cell_centres(lo[other], hi[other], Q)
            pts = np.empty((face.shape[0], d))
            pts[:, other] = face
            pts[:, axis] = hi[axis]
            tp = _features(centres[p], r, W[p], B0[p], pts)
            tq = _features(centres[qb], r, W[qb], B0[qb], pts)
            c0 = np.concatenate([tp, -tq], axis=1)
            dp = (1.0 - tp * tp) * (W[p][:, axis] / r)[None, :]
            dq = (1.0 - tq * tq) * (W[qb][:, axis] / r)[None, :]
            c1 = np.concatenate([dp, -dq], axis=1)
            P = pts.shape[0]
            vals = np.empty((2 * P, 2 * J))
            vals[0::2] = c0
            vals[1::2] = c1
            cols_row = np.concatenate([p * J + np.arange(J), qb * J + np.arange(J)]).astype(np.int64)
            cols = np.broadcast_to(cols_row, vals.shape)
            add(cols, vals, np.zeros((len(modes), 2 * P)))
            counts["interface"] += 2 * P

    row_nnz = np.concatenate([np.full(c.shape[0], c.shape[1], dtype=np.int64) for c in blocks_cols])
    m = row_nnz.shape[0]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(row_nnz, out=row_ptr[1:])
    col = np.concatenate([c.reshape(-1) for c in blocks_cols]).astype(np.int32)
    val = np.concatenate([v.reshape(-1) for v in blocks_vals]).astype(np.float64)
    b = np.ascontiguousarray(np.concatenate(rhs, axis=1))
    return RFMSystem(d=d, N=N, J=J, Q=Q, m=m, n=n, row_ptr=row_ptr, col=col, val=val, b=b,
                     modes=modes, centres=centres, radius=r, W=W, B0=B0, counts=counts, pde=pde,
                     kwave=kwave)


def build_config(name: str, modes=(1,)) -> tuple[RFMSystem, int]:
    """Return (system, s) for a named workload; s = gamma * n sketch rows."""
    c = CONFIGS[name]
    sysm = poisson_system(c["d"], c["N"], c["J"], c["Q"], modes=modes, pde=c.get("pde", "poisson"),
                          kwave=c.get("kwave", 0.0))
    return sysm, int(c["gamma"] * sysm.n)


def sample_points(d: int, npts: int = 10_000, seed: int = SAMPLE_POINT_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((npts, d))


def feature_eval(sysm: RFMSystem, pts: np.ndarray):
    """CSR of E with u_h(p) = (E x)(p): each point is owned by one half-open box
    [c-r, c+r) (the last box along each axis is closed) and evaluates its J features."""
    N, J, d = sysm.N, sysm.J, sysm.d
    cell = np.minimum(np.floor(pts * N).astype(np.int64), N - 1)
    owner = np.zeros(pts.shape[0], dtype=np.int64)
    for a in range(d):
        owner = owner * N + cell[:, a]
    npts = pts.shape[0]
    vals = np.empty((npts, J))
    for q in np.unique(owner):
        sel = owner == q
        vals[sel] = _features(sysm.centres[q], sysm.radius, sysm.W[q], sysm.B0[q], pts[sel])
    cols = owner[:, None] * J + np.arange(J)[None, :]
    row_ptr = np.arange(npts + 1, dtype=np.int64) * J
    return row_ptr, cols.reshape(-1).astype(np.int32), vals.reshape(-1)
