"""Seeded synthetic scenarios: meshes, beds, initial and boundary data.

Everything here is input construction for the shallow-water step (mesh
points, node elevations, region-defined initial values, Manning n per cell,
boundary tags and hydrographs).  The finite-volume arithmetic itself lives in
two independent places that both consume a :class:`Scenario`: the FP64 oracle
and the HIP library.

Workloads follow the paper's test catalogue (Results section, Table of
benchmarks): a wet-bed dam break in a flat channel, a lake at rest over a bed
with dry islands, a large valley flood fed by an inflow hydrograph (standing
in for the paper's large hydrodynamic case, T1), the two-rarefaction problem
of T5 and the three-humps dam break of T6.  Random draws use
``numpy.random.Generator(PCG64(BASE_SEED + offset))``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
from scipy.spatial import cKDTree

from . import mesh as M

BASE_SEED = 210212862

# boundary kinds (mirrors the library's and the oracle's enums by value)
WALL = 0
INFLOW_UNIFORM = 1
OUTFLOW_ZEROGRAD = 2
ZHYDROGRAPH = 3   # prescribed water-surface elevation series (t, Q hold times and elevations)
INFLOW_FROUDE = 4     # discharge series entering at a given Froude number (slope = Fr)
OUTFLOW_UNIFORM = 5   # normal depth of the outflowing discharge (slope = energy slope)
OUTFLOW_WEIR = 6      # Poleni weir (slope = crest elevation, par = Poleni factor)
OUTFLOW_HQ = 7        # h-Q relation (t = surface elevations, Q = discharges)
DYNAMIC_WALL = 8      # wall until the collapse time (slope) or depth (par), then zero gradient


def rng(offset: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + offset))


@dataclasses.dataclass
class BC:
    tag: int
    kind: int
    slope: float = 0.0              # energy slope (uniform), Froude number, crest elevation (weir), collapse time
    t: Optional[np.ndarray] = None  # hydrograph times [s] (surface elevations [m] of an h-Q table)
    Q: Optional[np.ndarray] = None  # discharge [m^3/s] (surface elevation [m] for ZHYDROGRAPH)
    phi_in: tuple = ()              # inflow concentration of each passive species
    par: float = 0.0                # Poleni factor of a weir, collapse depth of a dynamic wall


# external water sources and sinks: modes and units of the series
SRC_EXACT, SRC_AVAILABLE, SRC_INFINITY = 0, 1, 2
SRC_DISCHARGE, SRC_INTENSITY = 0, 1


@dataclasses.dataclass
class Source:
    mode: int                       # SRC_EXACT (adds or removes), SRC_AVAILABLE or SRC_INFINITY (sinks)
    unit: int = SRC_DISCHARGE       # total discharge over the region [m^3/s] or intensity [mm/h]
    t: Optional[np.ndarray] = None  # series times [s] (none for SRC_INFINITY)
    v: Optional[np.ndarray] = None  # series values (negative: a sink)


@dataclasses.dataclass
class Morpho:
    """Exner module: sediment closure ("mpm", "grass" or "eh") with alpha,
    exponent m and threshold thr (theta_cr, or u_cr for grass), grain
    diameter d_m [m], relative density s_rel, porosity, and an optional
    non-erodible bed z_rel (<= 0) below the initial bed per cell."""
    closure: str = "mpm"
    alpha: float = 8.0
    m: float = 1.5
    thr: float = 0.047
    d_m: float = 1e-3
    s_rel: float = 2.65
    porosity: float = 0.4
    z_rel: Optional[np.ndarray] = None


@dataclasses.dataclass
class Diffusion:
    """Diffusion of the passive species: molecular diffusivity Km [m^2/s]
    (one value, or one per species), longitudinal and transversal dispersion
    coefficients alpha_L, alpha_T (scaled by h u_*, u_* = |u| / c_f), and
    the relaxation time zeta [s] of the hyperbolic (Cattaneo-type) form."""
    Km: object = 0.0
    alpha_L: float = 0.0
    alpha_T: float = 0.0
    zeta: float = 1.0


@dataclasses.dataclass
class Scenario:
    name: str
    nodes: np.ndarray            # (V,3) float64: x, y, bed elevation z
    tri: np.ndarray              # (N,3) int32
    bnd_seg: np.ndarray          # (S,2) int32 node pairs of tagged boundary edges
    bnd_tag: np.ndarray          # (S,) int32
    bcs: List[BC]
    H0: Optional[np.ndarray]     # (N,) water surface elevation (clamped to the bed)
    h0: Optional[np.ndarray]     # (N,) water depth (used when H0 is None)
    qx0: np.ndarray
    qy0: np.ndarray
    manning: np.ndarray          # (N,) friction parameter: Manning n [s m^-1/3] (or k_str, K_s, y_R)
    t_end: float
    g: float = 9.81
    cfl: float = 0.9
    h_min: float = 1e-4
    dt_max: float = float("inf")
    friction: str = "manning"    # closure the `manning` array parameterises: manning, strickler, chezy, bezzola
    phi0: Optional[np.ndarray] = None  # (S, N) initial concentrations of S <= 5 advected species
    diffusion: Optional[Diffusion] = None  # diffusion of the species (relaxation form)
    sources: tuple = ()                # external water sources and sinks (Source)
    src_region: Optional[np.ndarray] = None  # (N,) int32 index into sources, -1 for none
    morpho: Optional[Morpho] = None    # Exner module (bed evolution)
    drain: bool = False                # draining-time positivity limiter instead of the bare clip

    @property
    def n_cells(self) -> int:
        return int(self.tri.shape[0])

    def centroids(self) -> np.ndarray:
        return self.nodes[self.tri, :2].mean(axis=1)


def _no_segments():
    return np.zeros((0, 2), np.int32), np.zeros((0,), np.int32)


def _assemble(name, xy, z, tri, segs, bcs, H0=None, h0=None, qx0=None, qy0=None,
              manning=None, t_end=0.0, **kw) -> Scenario:
    n = tri.shape[0]
    if segs:
        bs = np.concatenate([s for s, _ in segs]).astype(np.int32)
        bt = np.concatenate([np.full(len(s), t, np.int32) for s, t in segs])
    else:
        bs, bt = _no_segments()
    return Scenario(
        name=name,
        nodes=np.c_[xy, z].astype(np.float64),
        tri=np.ascontiguousarray(tri, dtype=np.int32),
        bnd_seg=np.ascontiguousarray(bs.reshape(-1, 2)),
        bnd_tag=bt,
        bcs=list(bcs),
        H0=None if H0 is None else np.asarray(H0, np.float64),
        h0=None if h0 is None else np.asarray(h0, np.float64),
        qx0=np.zeros(n) if qx0 is None else np.asarray(qx0, np.float64),
        qy0=np.zeros(n) if qy0 is None else np.asarray(qy0, np.float64),
        manning=np.zeros(n) if manning is None else np.asarray(manning, np.float64),
        t_end=float(t_end),
        **kw,
    )


# ---------------------------------------------------------------- dam break
def dam_break(d: float = 1.0, h_right: float = 0.1, t_end: float = 5.0) -> Scenario:
    """100 m x 10 m flat frictionless channel of right triangles with legs d,
    water at 1.0 m left of x=50 m and ``h_right`` to the right, at rest, all
    walls, CFL 0.9.  ``h_right=0.1`` is the wet-bed (Stoker) case and
    ``h_right=0`` the dry-bed (Ritter) case."""
    xy, tri, _ = M.structured_right(100.0, 10.0, d)
    cx = xy[tri, 0].mean(axis=1)
    h0 = np.where(cx < 50.0, 1.0, h_right)
    return _assemble(f"dam_break_d{d}", xy, np.zeros(len(xy)), tri, [], [],
                     h0=h0, t_end=t_end, cfl=0.9)


# ------------------------------------------------------------ lake at rest
def gaussian_bumps(xy: np.ndarray, lx: float, ly: float, r: np.random.Generator, n: int = 40):
    c = np.c_[r.uniform(0, lx, n), r.uniform(0, ly, n)]
    a = r.uniform(0.2, 2.5, n)
    s = r.uniform(20.0, 150.0, n)
    z = np.zeros(len(xy))
    for k in range(n):
        d2 = ((xy - c[k]) ** 2).sum(axis=1)
        z += a[k] * np.exp(-d2 / (2 * s[k] ** 2))
    return z


def lake_at_rest(n_cells: int = 200_000, seed: int = 0, lx: float = 2000.0,
                 ly: float = 1000.0, level: float = 1.5, t_end: float = 600.0) -> Scenario:
    """Delaunay mesh of seeded random points with every angle above 28
    degrees, bed = 40 seeded Gaussian bumps (0.2-2.5 m high, sigma 20-150 m),
    still water at ``level`` so bump tops are dry islands, Manning 0.035, walls."""
    xy, tri, _ = M.poisson_delaunay(lx, ly, n_cells, rng(1 + seed))
    z = gaussian_bumps(xy, lx, ly, rng(2 + seed))
    n = tri.shape[0]
    return _assemble(f"lake_at_rest_{n}", xy, z, tri, [], [], H0=np.full(n, level),
                     manning=np.full(n, 0.035), t_end=t_end, cfl=0.9)


# ------------------------------------------------------- level-boundary basin
def level_basin(times, levels, H0, d: float = 1.0, lx: float = 40.0, ly: float = 20.0,
                n: float = 0.02, t_end: float = 60.0, cfl: float = 0.5) -> Scenario:
    """Rectangle of right triangles (legs d) with a Gaussian mound (0.8 m
    high, at the centre) on a bed rising 1 mm/m in x, walls except the x = 0
    side, where the water-surface elevation follows (times, levels); the
    initial surface is H0 (dry where below the bed).  CFL 0.5: on right
    triangles the time step of eq. CFL_condition is unstable above about 0.6."""
    xy, tri, sides = M.structured_right(lx, ly, d)
    z = 0.8 * np.exp(-((xy[:, 0] - 0.5 * lx) ** 2 + (xy[:, 1] - 0.5 * ly) ** 2) / 30.0) + 1e-3 * xy[:, 0]
    segs = [(M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), 1)]
    bcs = [BC(1, ZHYDROGRAPH, t=np.asarray(times, np.float64), Q=np.asarray(levels, np.float64))]
    ntri = tri.shape[0]
    return _assemble(f"level_basin_{ntri}", xy, z, tri, segs, bcs, H0=np.full(ntri, H0),
                     manning=np.full(ntri, n), t_end=t_end, cfl=cfl)


# ------------------------------------------------------------ valley flood
def _fractal_noise(lx, ly, r: np.random.Generator, rms=0.5, spacing=10.0, beta=3.6):
    nx = int(2 ** np.ceil(np.log2(max(8, lx / spacing))))
    ny = int(2 ** np.ceil(np.log2(max(8, ly / spacing))))
    kx = np.fft.fftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    k = np.sqrt(kx ** 2 + ky ** 2)
    k[0, 0] = np.inf
    amp = k ** (-beta / 2.0)
    phase = r.uniform(0, 2 * np.pi, size=(ny, nx))
    field = np.real(np.fft.ifft2(amp * np.exp(1j * phase)))
    field *= rms / field.std()
    gx = np.linspace(0, lx, nx)
    gy = np.linspace(0, ly, ny)
    return gx, gy, field


def _bilinear(gx, gy, f, x, y):
    fx = np.clip((x - gx[0]) / (gx[1] - gx[0]), 0, len(gx) - 1 - 1e-9)
    fy = np.clip((y - gy[0]) / (gy[1] - gy[0]), 0, len(gy) - 1 - 1e-9)
    i = fx.astype(np.int64)
    j = fy.astype(np.int64)
    tx = fx - i
    ty = fy - j
    return ((1 - tx) * (1 - ty) * f[j, i] + tx * (1 - ty) * f[j, i + 1]
            + (1 - tx) * ty * f[j + 1, i] + tx * ty * f[j + 1, i + 1])


def centreline(lx: float, y0: float, wavelength: float = 1200.0, amp: float = 1.0, ds: float = 1.0):
    """Sine-generated meander: heading theta(s) = amp*sin(2 pi s / wavelength),
    starting at (0, y0) toward +x, integrated until it leaves x = lx."""
    pts = [(0.0, y0)]
    x, y, s = 0.0, y0, 0.0
    while x <= lx + ds:
        th = amp * np.sin(2 * np.pi * (s + 0.5 * ds) / wavelength)
        x += ds * np.cos(th)
        y += ds * np.sin(th)
        s += ds
        pts.append((x, y))
    return np.asarray(pts)


def valley_flood(n_cells: int = 4_000_000, seed: int = 0, scale: float = 1.0,
                 snapshot: Optional[str] = None, t_end: float = 3600.0,
                 q_peak: float = 2000.0, t_rise: float = 3600.0) -> Scenario:
    """Synthetic valley: DEM z = 20 - 1e-3 x + fractal noise (0.5 m RMS,
    spectrum k^-3.6) - 3 m inside a 40 m wide meandering channel, on a
    Delaunay mesh of a jittered lattice over (20 km x 4 km) * ``scale``.
    Manning n uniform in [0.025, 0.06] per 100 m patch.  Inflow uniform(Q,
    S=1e-3) on the channel mouth at x=0 with Q rising 50 -> ``q_peak`` over
    ``t_rise``; zero-gradient outflow at the far end; walls elsewhere.

    ``snapshot=None`` starts dry (H = z).  ``snapshot="wet"`` starts with 1 m
    of water moving at 0.5 m/s along x everywhere, so every cell does the full
    work of a step."""
    lx, ly = 20000.0 * scale, 4000.0 * scale
    xy, tri, sides = M.jittered_lattice(lx, ly, max(16, n_cells // 2), rng(3 + seed))
    gx, gy, f = _fractal_noise(lx, ly, rng(4 + seed))
    yc = ly / 2.0
    cl = centreline(lx, yc)
    dist, _ = cKDTree(cl).query(xy)
    chan = (dist <= 20.0).astype(np.float64)
    z = 20.0 - 1e-3 * xy[:, 0] + _bilinear(gx, gy, f, xy[:, 0], xy[:, 1]) - 3.0 * chan
    n = tri.shape[0]
    c = xy[tri].mean(axis=1)
    px, py = int(np.ceil(lx / 100.0)), int(np.ceil(ly / 100.0))
    table = rng(5 + seed).uniform(0.025, 0.06, size=(py, px))
    manning = table[np.minimum((c[:, 1] // 100).astype(int), py - 1),
                    np.minimum((c[:, 0] // 100).astype(int), px - 1)]
    inflow = M.segments_on_side(xy, sides["x0"], yc - 20.0, yc + 20.0, axis=1)
    outflow = M.segments_on_side(xy, sides["x1"], -1.0, ly + 1.0, axis=1)
    bcs = [BC(1, INFLOW_UNIFORM, slope=1e-3, t=np.array([0.0, t_rise]), Q=np.array([50.0, q_peak])),
           BC(2, OUTFLOW_ZEROGRAD)]
    if snapshot == "wet":
        h0, qx0 = np.ones(n), np.full(n, 0.5)
    else:
        h0, qx0 = np.zeros(n), np.zeros(n)
    return _assemble(f"valley_flood_{n}" + (f"_{snapshot}" if snapshot else ""), xy, z, tri,
                     [(inflow, 1), (outflow, 2)], bcs, h0=h0, qx0=qx0,
                     manning=manning, t_end=t_end, cfl=0.9)


def wet_snapshot(sc: Scenario) -> Scenario:
    """The fully wet snapshot of a valley-flood scenario on the same mesh:
    1 m of water moving at 0.5 m/s along x everywhere."""
    n = sc.n_cells
    name = sc.name if sc.name.endswith("_wet") else sc.name + "_wet"
    return Scenario(**{**sc.__dict__, "name": name, "H0": None, "h0": np.ones(n), "qx0": np.full(n, 0.5),
                       "qy0": np.zeros(n)})


# --------------------------------------------------------- batched ensemble
def ensemble_sizes(k: int = 64, lo: float = 2e4, hi: float = 5e5) -> np.ndarray:
    return np.round(np.exp(rng(7).uniform(np.log(lo), np.log(hi), k))).astype(np.int64)


def ensemble_member(k: int, n_cells: int, t_end: float = 1800.0, mesh: str = "poisson") -> Scenario:
    """One member of the batched ensemble: the lake-at-rest generator with
    its own seed, fed through x=0, y in [450,550] by Q_k(t) = 50 + (P_k-50)
    t/1800 with P_k ~ U[200,3000], zero-gradient outflow at x=2000.
    ``mesh="lattice"`` swaps the 28-degree Poisson-disk mesh for the faster
    jittered-lattice Delaunay mesh (same bed, same boundaries)."""
    lx, ly = 2000.0, 1000.0
    if mesh == "lattice":
        xy, tri, sides = M.jittered_lattice(lx, ly, max(16, n_cells // 2), rng(100 + k))
    else:
        xy, tri, sides = M.poisson_delaunay(lx, ly, n_cells, rng(100 + k))
    z = gaussian_bumps(xy, lx, ly, rng(2 + 100 + k))
    n = tri.shape[0]
    p = rng(200 + k).uniform(200.0, 3000.0)
    inflow = M.segments_on_side(xy, sides["x0"], 450.0, 550.0, axis=1)
    outflow = M.segments_on_side(xy, sides["x1"], -1.0, ly + 1.0, axis=1)
    bcs = [BC(1, INFLOW_UNIFORM, slope=1e-3, t=np.array([0.0, 1800.0]), Q=np.array([50.0, p])),
           BC(2, OUTFLOW_ZEROGRAD)]
    return _assemble(f"ensemble_{k}_{n}", xy, z, tri, [(inflow, 1), (outflow, 2)], bcs,
                     H0=np.full(n, 1.5), manning=np.full(n, 0.035), t_end=t_end, cfl=0.9)


# ------------------------------------------------------------------ serving
def serving_trace(n_requests: int = 512, rate: float = 4.0, n_lo: float = 1e4,
                  n_hi: float = 2e6, h_lo: float = 60.0, h_hi: float = 1800.0):
    """Poisson arrivals (exponential gaps at ``rate`` per second), mesh sizes
    log-uniform in [n_lo, n_hi], horizons uniform in [h_lo, h_hi] seconds."""
    r = rng(6)
    gaps = r.exponential(1.0 / rate, n_requests)
    arrive = np.cumsum(gaps) - gaps[0]
    sizes = np.round(np.exp(r.uniform(np.log(n_lo), np.log(n_hi), n_requests))).astype(np.int64)
    horizon = r.uniform(h_lo, h_hi, n_requests)
    return arrive, sizes, horizon


def serving_request(i: int, n_cells: int, horizon: float) -> Scenario:
    """A valley-flood request whose domain is scaled by sqrt(N/4e6) so the
    cell size (about 20 m^2) and time step stay those of the full valley."""
    s = float(np.sqrt(n_cells / 4e6))
    sc = valley_flood(n_cells=n_cells, seed=1000 + i, scale=s, t_end=horizon, t_rise=horizon)
    sc.name = f"request_{i}_{sc.n_cells}"
    return sc


def serving_pool(n_pool: int = 12, n_lo: float = 1e4, n_hi: float = 2e6) -> np.ndarray:
    """Mesh sizes of a cached pool of serving domains: log-spaced over
    [n_lo, n_hi], so a request drawn log-uniformly finds a pool mesh within a
    factor (n_hi/n_lo)^(1/(2(n_pool-1))) of its size."""
    return np.round(np.exp(np.linspace(np.log(n_lo), np.log(n_hi), n_pool))).astype(np.int64)


def pool_request(base: Scenario, rid: int, horizon: float) -> Scenario:
    """A request on a pooled serving domain: the domain's mesh and bed with
    its own horizon, the inflow hydrograph rising over that horizon."""
    bcs = []
    for b in base.bcs:
        if b.kind == INFLOW_UNIFORM:
            b = dataclasses.replace(b, t=np.array([0.0, horizon]), Q=np.asarray(b.Q, np.float64).copy())
        bcs.append(b)
    return Scenario(**{**base.__dict__, "name": f"request_{rid}_{base.n_cells}", "bcs": bcs,
                       "t_end": float(horizon)})


# ------------------------------------------------- paper T5 / T6 (hydro part)
def t5_rarefactions(d: float = 0.1, t_end: float = 2.5) -> Scenario:
    """T5 hydrodynamics: flat 100 m x 0.1 m channel, h = 1 m, q_x = -3 m^2/s
    left of x = 50 m and +3 m^2/s right of it, transmissive ends (zero
    gradient), reflective sides, CFL 0.95."""
    xy, tri, sides = M.structured_right(100.0, 0.1 if d <= 0.1 else d, d)
    cx = xy[tri, 0].mean(axis=1)
    n = tri.shape[0]
    qx = np.where(cx < 50.0, -3.0, 3.0)
    segs = [(M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), 2),
            (M.segments_on_side(xy, sides["x1"], -1, 1e9, 1), 2)]
    phi = np.where(cx < 50.0, 1.0, 0.0)[None, :]   # one advected species
    return _assemble(f"t5_d{d}", xy, np.zeros(len(xy)), tri, segs,
                     [BC(2, OUTFLOW_ZEROGRAD)], h0=np.ones(n), qx0=qx, t_end=t_end, cfl=0.95,
                     phi0=phi)


def t6_bed(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    e1 = 1.0 - np.sqrt((x - 30.0) ** 2 + (y + 9.0) ** 2) / 8.0
    e2 = 1.0 - np.sqrt((x - 30.0) ** 2 + (y - 9.0) ** 2) / 8.0
    e3 = 3.0 - 0.3 * np.sqrt((x - 47.5) ** 2 + y ** 2)
    return np.maximum.reduce([np.zeros_like(x), e1, e2, e3])


def t6_three_humps(n_cells: int = 20_000, t_end: float = 1200.0, seed: int = 0) -> Scenario:
    """T6 hydrodynamics: [0,75] x [-15,15] m, bed max(0, eta1, eta2, eta3),
    water surface 1.0 m for x < 16 m and 0.125 m elsewhere (the second value
    read as a surface elevation, so humps above it start dry), at rest,
    Manning 0.01, walls, CFL 0.95."""
    xy, tri, _ = M.poisson_delaunay(75.0, 30.0, n_cells, rng(20 + seed))
    xy = xy.copy()
    xy[:, 1] -= 15.0
    z = t6_bed(xy[:, 0], xy[:, 1])
    cx = xy[tri, 0].mean(axis=1)
    n = tri.shape[0]
    H0 = np.where(cx < 16.0, 1.0, 0.125)
    # two species: 0.5 / 0 left of the dam, 0 / 0.1 right of it (advected;
    # the paper also diffuses them with K = 0.25 m^2/s)
    phi = np.stack([np.where(cx < 16.0, 0.5, 0.0), np.where(cx < 16.0, 0.0, 0.1)])
    return _assemble(f"t6_{n}", xy, z, tri, [], [], H0=H0, manning=np.full(n, 0.01),
                     t_end=t_end, cfl=0.95, phi0=phi)


# ------------------------------------------------------------ tiny meshes
def tiny_random(nx: int = 2, ny: int = 2, seed: int = 0, dry_frac: float = 0.3,
                bcs: bool = True) -> Scenario:
    """A few right triangles (2*nx*ny cells) with a random bed and random
    wet/dry states and discharges; optional inflow on x=0 and zero-gradient
    outflow on x=1.  Some triangles are given clockwise to exercise the
    orientation fix."""
    r = rng(50 + seed)
    xy, tri, sides = M.structured_right(float(nx), float(ny), 1.0)
    xy = xy + np.c_[r.uniform(-0.15, 0.15, len(xy)), r.uniform(-0.15, 0.15, len(xy))] * \
        np.c_[(xy[:, 0] > 0) & (xy[:, 0] < nx), (xy[:, 1] > 0) & (xy[:, 1] < ny)]
    z = r.uniform(0.0, 0.5, len(xy))
    n = tri.shape[0]
    tri = tri.copy()
    flip = r.random(n) < 0.3
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    h0 = r.uniform(0.05, 1.0, n) * (r.random(n) > dry_frac)
    qx = r.uniform(-0.5, 0.5, n) * (h0 > 0)
    qy = r.uniform(-0.5, 0.5, n) * (h0 > 0)
    manning = r.uniform(0.0, 0.05, n)
    segs, bl = [], []
    if bcs:
        segs = [(M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), 1),
                (M.segments_on_side(xy, sides["x1"], -1, 1e9, 1), 2)]
        bl = [BC(1, INFLOW_UNIFORM, slope=1e-3, t=np.array([0.0, 10.0]), Q=np.array([0.2, 0.6])),
              BC(2, OUTFLOW_ZEROGRAD)]
        manning = np.maximum(manning, 0.01)
    return _assemble(f"tiny_{nx}x{ny}_{seed}", xy, z, tri, segs, bl, h0=h0, qx0=qx, qy0=qy,
                     manning=manning, t_end=1.0, cfl=0.9)
