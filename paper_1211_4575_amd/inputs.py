"""Seeded synthetic inputs (particle loaders) shared by the oracle tests and the GPU path.

This module holds no arithmetic of the particle-in-cell method itself: it only
draws positions and momenta.  Random numbers come from Philox-4x32-10 (Salmon,
Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), a
counter-based generator, so any particle's draws depend only on
(seed, stream, particle index, draw index) -- independent of how the load is
split, which is the property the paper asks of its generators (Sec. V.A).

Loaders follow the workloads in the design notes: pair loading so that the
initial charge density vanishes (Sec. V.A: particles injected in pairs of
opposite charge), quiet lattice loading of electron beams over a fixed ion
background, drifting Maxwellians with per-component spread u_th of the proper
velocity, and Maxwell-Juettner momenta by Sobol's rejection method
(Sobol 1976, as described by Zenitani 2015).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12114575

# Philox-4x32 constants (Salmon et al. 2011): round multipliers and Weyl key increments.
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = np.uint32(0x9E3779B9)
_PHILOX_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox-4x32-R block function on uint32 arrays; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = np.uint32(k0 + _PHILOX_W0)
                k1 = np.uint32(k1 + _PHILOX_W1)
            p0 = _PHILOX_M0 * c0.astype(np.uint64)
            p1 = _PHILOX_M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _u53(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Two uint32 words -> float64 uniform strictly inside (0, 1) (53 random bits, centred)."""
    hi = (a >> np.uint32(5)).astype(np.float64)  # 27 bits
    lo = (b >> np.uint32(6)).astype(np.float64)  # 26 bits
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 9007199254740992.0)


def uniforms(seed: int, stream: int, index: np.ndarray, ndraw: int) -> np.ndarray:
    """``ndraw`` uniforms in (0,1) for each particle index: array [ndraw, len(index)].

    Counter = (index low word, index high word, block, stream); key = (seed low, seed high).
    Each Philox block yields two uniforms.
    """
    index = np.asarray(index, dtype=np.uint64)
    lo = (index & _MASK32).astype(np.uint32)
    hi = (index >> np.uint64(32)).astype(np.uint32)
    out = np.empty((ndraw, index.size), dtype=np.float64)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    for blk in range((ndraw + 1) // 2):
        r0, r1, r2, r3 = philox4x32(lo, hi, np.uint32(blk), np.uint32(stream), k0, k1)
        out[2 * blk] = _u53(r0, r1)
        if 2 * blk + 1 < ndraw:
            out[2 * blk + 1] = _u53(r2, r3)
    return out


def normals(seed: int, stream: int, index: np.ndarray, ndraw: int) -> np.ndarray:
    """Standard normals by Box-Muller from :func:`uniforms`: array [ndraw, len(index)]."""
    nu = ndraw + (ndraw & 1)
    U = uniforms(seed, stream, index, nu)
    out = np.empty((nu, U.shape[1]))
    for p in range(0, nu, 2):
        r = np.sqrt(-2.0 * np.log(U[p]))
        th = 2.0 * math.pi * U[p + 1]
        out[p] = r * np.cos(th)
        out[p + 1] = r * np.sin(th)
    return out[:ndraw]


def maxwell_juttner_speed(seed: int, stream: int, index: np.ndarray, theta: float, max_tries: int = 64):
    """Proper-speed magnitude |u| / c of a Maxwell-Juettner distribution at kT/mc^2 = theta,
    by Sobol's rejection: u = -theta ln(X1 X2 X3), eta = -theta ln(X1 X2 X3 X4),
    accept when eta^2 - u^2 > 1.  Attempt t uses draw block 2t, 2t+1 (uniforms 4t..4t+3).
    """
    index = np.asarray(index, dtype=np.uint64)
    out = np.full(index.size, np.nan)
    todo = np.arange(index.size)
    for t in range(max_tries):
        if todo.size == 0:
            break
        U = _uniform_block(seed, stream, index[todo], 2 * t, 2)
        x1, x2, x3, x4 = U
        u = -theta * np.log(x1 * x2 * x3)
        eta = -theta * np.log(x1 * x2 * x3 * x4)
        ok = eta * eta - u * u > 1.0
        out[todo[ok]] = u[ok]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("Maxwell-Juttner sampler did not accept within max_tries")
    return out


def _uniform_block(seed, stream, index, first_block, nblocks):
    lo = (index & _MASK32).astype(np.uint32)
    hi = (index >> np.uint64(32)).astype(np.uint32)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    outs = []
    for blk in range(first_block, first_block + nblocks):
        r0, r1, r2, r3 = philox4x32(lo, hi, np.uint32(blk), np.uint32(stream), k0, k1)
        outs.append(_u53(r0, r1))
        outs.append(_u53(r2, r3))
    return outs


def isotropic_directions(seed, stream, index):
    """Unit vectors uniform on the sphere: [3, n]."""
    U = uniforms(seed, stream, index, 2)
    cz = 2.0 * U[0] - 1.0
    ph = 2.0 * math.pi * U[1]
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz])


# ---------------------------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------------------------
@dataclass
class Species:
    name: str
    q: float
    m: float
    w: float
    pos: np.ndarray  # [3, n] float64, cell units in [0, N)
    u: np.ndarray  # [3, n] float64 proper velocity


@dataclass
class Workload:
    name: str
    n: tuple  # cells (nx, ny, nz)
    d: tuple  # cell sizes
    dt: float
    shape_order: int
    field_order: int
    species: list = field(default_factory=list)
    rho_background: float = 0.0
    alpha: float = 0.55
    pusher: int = 0
    steps: int = 1

    def params(self, **over):
        p = dict(n=self.n, d=self.d, dt=self.dt, c=1.0, eps0=1.0, shape_order=self.shape_order,
                 field_order=self.field_order, alpha=self.alpha, pusher=self.pusher,
                 relax_tol=1e-14, relax_max_iter=200, rho_background=self.rho_background)
        p.update(over)
        return p

    @property
    def n_particles(self):
        return sum(s.pos.shape[1] for s in self.species)


# stream ids: (workload << 8) | (species << 4) | purpose
def _stream(wl: int, sp: int, purpose: int) -> int:
    return (wl << 8) | (sp << 4) | purpose


def uniform_positions(seed, stream, n_part, n_cells):
    idx = np.arange(n_part, dtype=np.uint64)
    U = uniforms(seed, stream, idx, 3)
    pos = np.empty((3, n_part))
    for d in range(3):
        pos[d] = U[d] * n_cells[d]
        pos[d] = np.where(pos[d] >= n_cells[d], 0.0, pos[d])
    return pos


def lattice_positions(n_cells, per_dim):
    """Quiet start: per_dim = (kx, ky, kz) particles per cell per dimension on a regular lattice
    at offsets (a + 1/2)/k.  B-spline weights of any order deposit an exactly uniform density
    from such a lattice (sum of integer shifts of a B-spline is one)."""
    axes = []
    for d in range(3):
        k = per_dim[d]
        axes.append((np.arange(n_cells[d] * k, dtype=np.float64) + 0.5) / k)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


def thermal_u(seed, stream, n_part, uth, drift=(0.0, 0.0, 0.0)):
    idx = np.arange(n_part, dtype=np.uint64)
    G = normals(seed, stream, idx, 3)
    return np.stack([drift[d] + uth * G[d] for d in range(3)])


def plain_heating(seed=SEED_BASE, n=(16, 16, 16), ppc=8, uth=0.1, shape_order=2, field_order=2, dt=0.4):
    """Plain-method FP64 workload: electrons and positrons, pair-loaded at uniform-random
    positions (zero initial charge density), Maxwellian proper velocities, zero fields."""
    npart = n[0] * n[1] * n[2] * ppc
    pos = uniform_positions(seed, _stream(1, 0, 0), npart, n)
    ue = thermal_u(seed, _stream(1, 0, 1), npart, uth)
    up = thermal_u(seed, _stream(1, 1, 1), npart, uth)
    w = 1.0 / ppc
    sp = [Species("electron", -1.0, 1.0, w, pos, ue), Species("positron", 1.0, 1.0, w, pos.copy(), up)]
    return Workload("plain_heating", tuple(n), (1.0, 1.0, 1.0), dt, shape_order, field_order, sp, steps=100)


def two_stream(seed=SEED_BASE, n=(128, 32, 32), per_dim=(4, 4, 2), v_beam=0.2, uth=0.01, dx=0.1,
               shape_order=3, field_order=6, cfl=0.4, wl_id=2):
    """Two counter-streaming electron beams along x over a fixed neutralising ion background.
    Quiet lattice loading of both beams at the same points (density exactly uniform, so the
    initial E is zero); thermal spread uth per component seeds the instability."""
    ppc = per_dim[0] * per_dim[1] * per_dim[2]
    pos = lattice_positions(n, per_dim)
    npart = pos.shape[1]
    g0 = 1.0 / math.sqrt(1.0 - v_beam * v_beam)
    u1 = thermal_u(seed, _stream(wl_id, 0, 1), npart, uth, (+v_beam * g0, 0.0, 0.0))
    u2 = thermal_u(seed, _stream(wl_id, 1, 1), npart, uth, (-v_beam * g0, 0.0, 0.0))
    w = 0.5 / ppc
    sp = [Species("beam+", -1.0, 1.0, w, pos, u1), Species("beam-", -1.0, 1.0, w, pos.copy(), u2)]
    return Workload("two_stream", tuple(n), (dx, dx, dx), cfl * dx, shape_order, field_order, sp,
                    rho_background=1.0, steps=2000)


def pair_maxwell_juttner(seed=SEED_BASE, n=(256, 256, 256), ppc=32, theta=1.0, shape_order=3,
                         field_order=6, dt=0.4, index_range=None):
    """Relativistic pair plasma, Maxwell-Juettner at kT = theta m c^2, pair-loaded.
    ``index_range`` = (start, stop) loads only that slice of the particle list (same values
    as the full load at those indices)."""
    npart = n[0] * n[1] * n[2] * ppc
    lo, hi = (0, npart) if index_range is None else index_range
    idx = np.arange(lo, hi, dtype=np.uint64)
    U = uniforms(seed, _stream(3, 0, 0), idx, 3)
    pos = np.stack([np.where(U[d] * n[d] >= n[d], 0.0, U[d] * n[d]) for d in range(3)])
    sp = []
    for s, (nm, q) in enumerate((("electron", -1.0), ("positron", 1.0))):
        mag = maxwell_juttner_speed(seed, _stream(3, s, 1), idx, theta)
        dirs = isotropic_directions(seed, _stream(3, s, 2), idx)
        sp.append(Species(nm, q, 1.0, 1.0 / ppc, pos.copy(), dirs * mag))
    return Workload("pair_mj", tuple(n), (1.0, 1.0, 1.0), dt, shape_order, field_order, sp, steps=200)


def kelvin_helmholtz(seed=SEED_BASE, n=(1024, 512, 1), ppc=64, mass_ratio=25.0, v0=0.2, width=8.0,
                     uth=0.02, shape_order=3, field_order=6, dt=0.4):
    """Quasi-2D shear flow: two tanh shear layers at y = Ly/4 and 3Ly/4, bulk flow +-v0 along x
    for electrons and ions alike (no current), ions co-located with electrons (no charge)."""
    npart = n[0] * n[1] * n[2] * ppc
    pos = uniform_positions(seed, _stream(4, 0, 0), npart, n)
    Ly = float(n[1])
    y = pos[1]
    vx = v0 * (np.tanh((y - Ly / 4) / width) - np.tanh((y - 3 * Ly / 4) / width) - 1.0)
    g = 1.0 / np.sqrt(1.0 - vx * vx)
    sp = []
    for s, (nm, q, m) in enumerate((("electron", -1.0, 1.0), ("ion", 1.0, mass_ratio))):
        uu = thermal_u(seed, _stream(4, s, 1), npart, uth)
        uu[0] += vx * g
        sp.append(Species(nm, q, m, 1.0 / ppc, pos.copy(), uu))
    return Workload("kelvin_helmholtz", tuple(n), (1.0, 1.0, 1.0), dt, shape_order, field_order, sp, steps=5000)


def boost_z(u, gamma_b):
    """Four-velocities u (rest frame of a population, [3, n]) seen in the frame where that
    population drifts along +z with Lorentz factor gamma_b: u_z' = G (u_z + beta gamma)."""
    if gamma_b == 1.0:
        return u
    beta = math.sqrt(1.0 - 1.0 / (gamma_b * gamma_b))
    g = np.sqrt(1.0 + (u * u).sum(axis=0))
    out = u.copy()
    out[2] = gamma_b * (u[2] + beta * g)
    return out


MMI_SPECIES = (("beam electron", -1.0, False, True), ("beam ion", 1.0, True, True),
               ("background electron", -1.0, False, False), ("background ion", 1.0, True, False))


def mmi(seed=SEED_BASE, n=(128, 128, 128), ppc=20, gamma_b=4.0, n_b=0.1, n_p=0.9, T_b=0.01, T_p=0.1,
        mass_ratio=1836.0, dx=0.1, cfl=0.4, shape_order=3, field_order=6, index_range=None, quiet=False,
        lattice=None):
    """Relativistic mixed-mode two-stream set-up (Sec. VI, relativistic two-stream test): a cold
    thin neutral beam (electrons and ions, density n_b, Lorentz factor gamma_b along +z) through
    a warm thick neutral background at rest (density n_p); each population's electrons and ions
    share their uniform-random positions, so the initial charge and current vanish and no
    field is loaded.  Thermal proper velocities are Gaussian with variance T/m per component in
    the population's rest frame (temperatures in units of m_e c^2), then boosted.  ppc particles
    per cell per species; species order: beam electron, beam ion, background electron,
    background ion.  ``index_range`` = (start, stop) loads that slice of every species.
    ``quiet``: a quiet start, particles 2k and 2k+1 of a species at the same position (the
    draws of index 2k) with opposite rest-frame thermal velocities, so that the thermal
    current of each pair cancels at the start and the fields grow from a lower noise floor.
    ``lattice`` = (px, py, pz) with px py pz = ppc: every population on a regular lattice
    instead, particle i at sub-lattice point i mod ppc of cell i div ppc (cells and points x
    fastest), points at ((a + 1/2) / px, (b + 1/2) / py, (c + 1/2) / pz) of the cell."""
    npart = n[0] * n[1] * n[2] * ppc
    lo, hi = (0, npart) if index_range is None else index_range
    idx = np.arange(lo, hi, dtype=np.uint64)
    draw = idx & ~np.uint64(1) if quiet else idx
    sign = np.where(idx & np.uint64(1), -1.0, 1.0) if quiet else np.ones(len(idx))
    pos = {}
    if lattice is not None:
        px, py, pz = lattice
        if px * py * pz != ppc:
            raise ValueError("lattice must hold ppc points per cell")
        i = idx.astype(np.int64)
        c, sub = i // ppc, i % ppc
        cell = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
        frac = ((sub % px + 0.5) / px, ((sub // px) % py + 0.5) / py, (sub // (px * py) + 0.5) / pz)
        lat = np.stack([cell[d] + frac[d] for d in range(3)]).astype(np.float64)
        pos = {0: lat, 1: lat}
    else:
        for pop in (0, 1):  # 0 beam, 1 background
            U = uniforms(seed, _stream(5, 2 * pop, 0), draw, 3)
            pos[pop] = np.stack([np.where(U[d] * n[d] >= n[d], 0.0, U[d] * n[d]) for d in range(3)])
    sp = []
    for s, (nm, q, ion, beam) in enumerate(MMI_SPECIES):
        m = mass_ratio if ion else 1.0
        T = T_b if beam else T_p
        G = normals(seed, _stream(5, s, 1), draw, 3) * sign
        u = boost_z(math.sqrt(T / m) * G, gamma_b if beam else 1.0)
        dens = n_b if beam else n_p
        sp.append(Species(nm, q, m, dens / ppc, pos[0 if beam else 1].copy(), u))
    return Workload("mmi", tuple(n), (dx, dx, dx), cfl * dx, shape_order, field_order, sp, steps=1500)


def mmi_rates(gamma_b=4.0, n_b=0.1, n_p=0.9):
    """Cold-beam growth rates (units of the total electron plasma frequency) of the oblique
    mixed mode, filamentation and two-stream branches for a thin beam (eqs. "mmigrowth",
    "figrowth", "tsigrowth"), with alpha read as the beam's share of the total density, and
    the angle of the MMI wave vector to the beam, which the paper gives as about 74 degrees.
    Returns dict(mmi, fi, tsi, theta_deg)."""
    alpha = n_b / (n_b + n_p)
    beta = math.sqrt(1.0 - 1.0 / (gamma_b * gamma_b))
    c = 2.0 ** (-4.0 / 3.0) * math.sqrt(3.0) * alpha ** (1.0 / 3.0)
    return dict(mmi=c * gamma_b ** (-1.0 / 3.0), fi=beta * math.sqrt(alpha / gamma_b), tsi=c / gamma_b,
                theta_deg=74.0)


# ---------------------------------------------------------------------------------------------
# Serving ensemble: a stream of small two-stream runs (a parameter scan)
# ---------------------------------------------------------------------------------------------
SERVING_GRIDS = ((32, 32, 32), (64, 32, 32), (128, 16, 16))
SERVING_LATTICES = ((2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4))  # 8, 16, 32, 64 per cell per beam


@dataclass
class TwoStreamRequest:
    """One request: a two-stream run (the loader :func:`two_stream` with these settings) of
    ``steps`` steps, arriving ``arrival`` seconds after the stream starts."""
    rid: int
    arrival: float
    n: tuple
    per_dim: tuple
    v_beam: float
    uth: float
    steps: int
    seed: int
    dx: float = 0.1
    cfl: float = 0.4
    wl_id: int = 5

    @property
    def ppc(self) -> int:
        return self.per_dim[0] * self.per_dim[1] * self.per_dim[2]

    @property
    def n_per_beam(self) -> int:
        return self.n[0] * self.n[1] * self.n[2] * self.ppc

    @property
    def updates(self) -> int:
        return 2 * self.n_per_beam * self.steps


def serving_requests(count=256, rate=1.0, seed=SEED_BASE, steps=(200, 2000), v_beam=(0.1, 0.5), uth=0.01,
                     grids=SERVING_GRIDS, lattices=SERVING_LATTICES):
    """Poisson stream of ``count`` two-stream requests at ``rate`` per second: grid and
    lattice uniform over the given sets, beam speed uniform in ``v_beam``, step count uniform
    over the integers in ``steps``; request i draws its particles with seed ``seed + 1 + i``."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    g = rng.integers(0, len(grids), count)
    lat = rng.integers(0, len(lattices), count)
    v = rng.uniform(v_beam[0], v_beam[1], count)
    k = rng.integers(steps[0], steps[1] + 1, count)
    return [TwoStreamRequest(i, float(t[i]), tuple(grids[g[i]]), tuple(lattices[lat[i]]), float(v[i]), float(uth),
                             int(k[i]), seed + 1 + i) for i in range(count)]


# ---------------------------------------------------------------------------------------------
# Split-precision form: integer cell (nearest cell centre) + in-cell offset in [-1/2, 1/2)
# ---------------------------------------------------------------------------------------------
def split_origin(shape_order: int) -> str:
    """Offset convention of the split form for a weight order: the nearest node (offset in
    [-1/2, 1/2)) for quadratic weights, the node below (offset in [0, 1)) for cubic weights,
    so that the centred support of every particle starts one node below its cell."""
    return "nearest" if shape_order == 2 else "floor"


def to_split(pos: np.ndarray, n, dtype=np.float32, origin="nearest"):
    """(cell linear index int32 x-fastest, offsets [3, n] in ``dtype``) of positions in [0, N),
    the cell being the nearest node (``origin="nearest"``, offset in [-1/2, 1/2)) or the node
    below (``origin="floor"``, offset in [0, 1)).  The offset is rounded to ``dtype``;
    :func:`from_split` gives the exactly represented position of that rounded state."""
    lo = {"nearest": -0.5, "floor": 0.0}[origin]
    ijk = np.floor(pos - lo)
    off = (pos - ijk).astype(dtype)
    # rounding can push an offset onto the upper end of the range; move such particles on
    bump = off >= dtype(lo + 1.0)
    ijk = ijk + bump
    # the moved particle sits a rounding error below the new cell's range: put it at its start
    off = np.where(bump, np.maximum((pos - ijk).astype(dtype), dtype(lo)), off)
    ijk = ijk.astype(np.int64)
    for d in range(3):
        ijk[d] %= n[d]
    cell = (ijk[0] + n[0] * (ijk[1] + n[1] * ijk[2])).astype(np.int32)
    return cell, off


def from_split(cell: np.ndarray, off: np.ndarray, n) -> np.ndarray:
    """Positions (float64, [0, N)) of a split state."""
    cell = cell.astype(np.int64)
    i = cell % n[0]
    j = (cell // n[0]) % n[1]
    k = cell // (n[0] * n[1])
    pos = np.stack([i, j, k]).astype(np.float64) + off.astype(np.float64)
    for d in range(3):
        pos[d] = np.mod(pos[d], n[d])
    return pos
