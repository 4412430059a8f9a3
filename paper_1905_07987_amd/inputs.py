"""Seeded synthetic inputs of the benchmark workloads.

Shared by the tests, the benchmark and the smoke check, and by both the HIP
path and the CPU oracle: each function maps node coordinates (from whichever
side asks) to an initial state, so both sides start from identical arrays.
Nothing here belongs to the ADER-DG method itself; the generators only define
workloads (shapes, value distributions, material layering, sources and
receivers).

Workloads
  c1  2-D Euler, N=3, 16x16 periodic cells on [0,1]^2: rho = 1 + 0.2 sin(2 pi (x+y)),
      u = v = 1, p = 1 (an exact travelling solution).
  c2  3-D Euler, N=5, 64^3 periodic cells on [0,1]^3: rho = 1 + 0.05 f_rho,
      p = 1 + 0.05 f_p, u = 0, f = (1/8) sum_{m<8} sin(2 pi k_m . x + phi_m) with
      k_m in {-3..3}^3 \\ {0} and phi_m ~ U[0, 2 pi), seed 7987.
  c3  3-D elasticity, N=4, 48^3 cells on [0, 24 km]^3, three horizontal layers
      (Table 3 of the paper for the top two), +-10 % per-cell perturbation,
      a Ricker point source (5 Hz) and 32 receivers, seed 7988.
  c4  3-D elasticity, N=3, 32^3 cells, same layering (seed 7989) and a
      +-5 % perturbed "observed" material (seed 7990).
  c5  3-D Euler, N=3, 96^3 cells on [0,1]^3 with reflecting walls, spherical
      explosion (seed 7991): inside a sphere of radius 0.2 with a random centre
      in [0.3, 0.7]^3 rho = 1, E = 1, outside rho = 0.125, E = 0.1, j = 0;
      run with the subcell limiter, the cells the sphere's surface crosses
      starting on FV with their subcell values sampled at the subcell centres.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def euler_conserved(rho, u, p, gamma=GAMMA):
    """(rho, rho u, E) with E = p/(gamma-1) + rho |u|^2 / 2, stacked on axis 1."""
    u = [np.asarray(ui) for ui in u]
    kin = sum(ui * ui for ui in u)
    E = p / (gamma - 1.0) + 0.5 * rho * kin
    return np.stack([rho] + [rho * ui for ui in u] + [E], axis=1)


def c1_state(xyz, t: float = 0.0):
    """[C][4][S] for node coordinates xyz[C][S][2]; exact at time t."""
    x, y = xyz[..., 0], xyz[..., 1]
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (x + y - 2.0 * t))
    return np.stack([rho, rho, rho, 2.5 + rho], axis=1)


def fourier_field(rng, xyz, modes: int = 8, kmax: int = 3):
    dim = xyz.shape[-1]
    ks = []
    while len(ks) < modes:
        k = rng.integers(-kmax, kmax + 1, size=dim)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    ph = rng.uniform(0.0, 2 * np.pi, size=modes)
    f = np.zeros(xyz.shape[:-1])
    for m in range(modes):
        f += np.sin(2 * np.pi * (xyz @ ks[m]) + ph[m])
    return f / modes


def c2_state(xyz, seed: int = 7987, amp: float = 0.05):
    """Smooth random Euler state: rho = 1 + amp f_rho, p = 1 + amp f_p, u = 0."""
    rng = np.random.default_rng(seed)
    frho = fourier_field(rng, xyz)
    fp = fourier_field(rng, xyz)
    dim = xyz.shape[-1]
    zero = np.zeros_like(frho)
    return euler_conserved(1.0 + amp * frho, [zero] * dim, 1.0 + amp * fp)


def smooth_euler_state(xyz, seed: int, amp: float = 0.2, vel: float = 0.3):
    """A smooth random Euler state with flow (used by the parity tests)."""
    rng = np.random.default_rng(seed)
    dim = xyz.shape[-1]
    rho = 1.0 + amp * fourier_field(rng, xyz, 4, 2)
    u = [vel * fourier_field(rng, xyz, 4, 2) for _ in range(dim)]
    p = 1.0 + amp * fourier_field(rng, xyz, 4, 2)
    return euler_conserved(rho, u, p)


def blast_state(xyz, seed: int = 7991, radius: float = 0.2):
    """The paper's circular/spherical explosion data with a random centre."""
    rng = np.random.default_rng(seed)
    dim = xyz.shape[-1]
    centre = rng.uniform(0.3, 0.7, size=dim)
    inside = ((xyz - centre) ** 2).sum(-1) < radius * radius
    rho = np.where(inside, 1.0, 0.125)
    E = np.where(inside, 1.0, 0.1)
    zero = np.zeros_like(rho)
    return np.stack([rho] + [zero] * dim + [E], axis=1)


def subcell_centres(cells, lo, hi, m: int):
    """[C][m^dim][dim] centres of the m^dim equal subcells of every cell
    (cells and subcells x fastest)."""
    dim = len(cells)
    h = [(hi[d] - lo[d]) / cells[d] for d in range(dim)]
    cidx = np.stack(np.meshgrid(*[np.arange(c) for c in cells[::-1]], indexing="ij")[::-1], -1).reshape(-1, dim)
    sidx = np.stack(np.meshgrid(*[np.arange(m)] * dim, indexing="ij")[::-1], -1).reshape(-1, dim)
    out = np.empty((len(cidx), len(sidx), dim))
    for d in range(dim):
        out[..., d] = lo[d] + (cidx[:, None, d] + (sidx[None, :, d] + 0.5) / m) * h[d]
    return out


def blast_limited_start(xyz_nodes, xyz_sub, seed: int = 7991, radius: float = 0.2):
    """The explosion data for a run with the subcell limiter, started along
    the discontinuity (the FV and DG subdomains initialised there): cells
    whose nodes or subcell centres lie on both sides of the sphere start on
    FV (status 3) with their subcell values sampled at the subcell centres.
    Returns (Q [C][nv][S] sampled at the nodes, sub [C][nv][m^dim] (zero
    outside the FV cells), status [C] uint8)."""
    Q = blast_state(xyz_nodes, seed, radius)
    sub = blast_state(xyz_sub, seed, radius)
    cut = lambda a: (a[:, 0].min(axis=1) != a[:, 0].max(axis=1))
    fv = cut(Q) | cut(sub)
    sub[~fv] = 0.0
    return Q, sub, np.where(fv, 3, 0).astype(np.uint8)


def blast_fv_cells(cells, lo, hi, order: int, seed: int = 7991, radius: float = 0.2):
    """The same start for meshes whose subcell centres do not all fit in
    host memory: the cells whose box the sphere's surface crosses start on
    FV, and only their subcells are sampled.  Returns (fv cell indices,
    sub [nfv][nv][m^dim] sampled at the subcell centres)."""
    rng = np.random.default_rng(seed)
    dim = len(cells)
    centre = rng.uniform(0.3, 0.7, size=dim)          # the draw of blast_state
    h = [(hi[d] - lo[d]) / cells[d] for d in range(dim)]
    grids = np.meshgrid(*[np.arange(c) for c in cells[::-1]], indexing="ij")[::-1]
    near = np.zeros(grids[0].shape)
    far = np.zeros(grids[0].shape)
    for d in range(dim):
        a = lo[d] + grids[d] * h[d] - centre[d]
        b = a + h[d]
        near += np.maximum(0.0, np.maximum(a, -b)) ** 2
        far += np.maximum(np.abs(a), np.abs(b)) ** 2
    fv = np.flatnonzero(((near < radius * radius) & (far > radius * radius)).ravel())
    m = 2 * order + 1
    sidx = np.stack(np.meshgrid(*[np.arange(m)] * dim, indexing="ij")[::-1], -1).reshape(-1, dim)
    cidx = np.stack([(fv // int(np.prod(cells[:d]))) % cells[d] for d in range(dim)], -1)
    xs = np.empty((len(fv), len(sidx), dim))
    for d in range(dim):
        xs[..., d] = lo[d] + (cidx[:, None, d] + (sidx[None, :, d] + 0.5) / m) * h[d]
    return fv, blast_state(xs, seed, radius)


# ----------------------------------------------------------------- elasticity
LAYERS_KM = ((0.0, 1.0, (4000.0, 2000.0, 2600.0)),    # Table 3, top layer
             (1.0, 12.0, (6000.0, 3464.0, 2700.0)),   # Table 3, half space
             (12.0, 1e9, (7000.0, 4000.0, 3000.0)))   # deeper layer (synthetic)


def layered_material(cell_centres_z_m, seed: int, perturb: float = 0.1):
    """Per-cell (rho, cp, cs) of the layered model with a seeded +-perturb
    multiplicative perturbation of each value.  Depth z is in metres."""
    zc = np.asarray(cell_centres_z_m) / 1000.0
    base = np.zeros((len(zc), 3))
    for lo, hi, (cp, cs, rho) in LAYERS_KM:
        m = (zc >= lo) & (zc < hi)
        base[m] = (rho, cp, cs)
    rng = np.random.default_rng(seed)
    return base * (1.0 + perturb * rng.uniform(-1.0, 1.0, size=base.shape))


def cell_centres(cells, lo, hi):
    cells = list(cells)
    h = [(hi[d] - lo[d]) / cells[d] for d in range(3)]
    cz, cy, cx = np.meshgrid(np.arange(cells[2]), np.arange(cells[1]), np.arange(cells[0]), indexing="ij")
    return np.stack([lo[0] + (cx.ravel() + 0.5) * h[0], lo[1] + (cy.ravel() + 0.5) * h[1],
                     lo[2] + (cz.ravel() + 0.5) * h[2]], axis=1)


def elastic_config(which: str = "c3"):
    """Mesh, material, source and receivers of the elastic workloads."""
    L = 24000.0
    if which == "c3":
        cells, order, seed, steps = (48, 48, 48), 4, 7988, 100
        src_x = (12250.0, 12250.0, 2250.0)
        rec = [(375.0 + 750.0 * r, 12250.0, 750.0) for r in range(32)]
    elif which == "c4":
        cells, order, seed, steps = (32, 32, 32), 3, 7989, 200
        src_x = (12375.0, 12375.0, 2625.0)
        rec = [(1125.0 + 1500.0 * r, 12375.0, 1125.0) for r in range(16)]
    else:
        raise ValueError(which)
    lo, hi = (0.0, 0.0, 0.0), (L, L, L)
    centres = cell_centres(cells, lo, hi)
    params = layered_material(centres[:, 2], seed)
    weight = [0.0] * 8 + [1.0]  # vertical body force on rho v_z
    source = dict(x=src_x, weight=weight, w=weight, f0=5.0, t0=0.2, amp=1.0)
    return dict(cells=cells, order=order, lo=lo, hi=hi, params=params, source=source,
                receivers=np.array(rec), steps=steps, seed=seed)


def elastic_zero_state(ncells: int, S: int):
    return np.zeros((ncells, 9, S))


def elastic_smooth_state(xyz, seed: int, scale_sigma: float = 5e3, scale_rhov: float = 1.0):
    """A smooth random elastic state for parity tests (units: Pa and kg/(m^2 s))."""
    rng = np.random.default_rng(seed)
    L = xyz.max() - xyz.min() + 1e-30
    fields = [scale_sigma * fourier_field(rng, xyz / L, 4, 2) for _ in range(6)]
    fields += [scale_rhov * fourier_field(rng, xyz / L, 4, 2) for _ in range(3)]
    return np.stack(fields, axis=1)
