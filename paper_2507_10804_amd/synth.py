"""Seeded synthetic inputs for the acoustic Gauss-Newton Hessian-vector product.

This module is shared by the HIP path, the tests, the bench and the oracle
drivers.  It draws models, perturbation vectors, acquisition geometry and the
source wavelet, and nothing else: it holds none of the method's arithmetic
(no stencil, sponge, recurrence, adjoint or reduction lives here).

Stand-ins for the paper's data (Section 4.2): the modified Marmousi model is
not available, so a seeded layered-and-faulted velocity model with the same
physical width (9.2 km) is generated instead; nothing of Marmousi is copied.

Every array is float64 and every generator takes an explicit seed
(``numpy.random.default_rng``, PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import gaussian_filter

# Maximum Courant number max(m)*dt/dx the leapfrog scheme tolerates with the
# 8th-order Laplacian used here (2/sqrt(2*6.5012)); inputs are generated well
# below it.
DEFAULT_CFL = 0.4


@dataclass
class Geometry:
    """Acquisition and discretisation of one wave-equation problem.

    Grid is nz rows (depth) by nx columns (horizontal, fastest axis), spacing
    dx in metres; nb absorbing cells are padded on every side.  Sources and
    receivers are (iz, ix) cells of the model grid.  ``wavelet`` holds s(n*dt)
    for n = 0..nt-1.
    """

    nx: int
    nz: int
    dx: float
    dt: float
    nt: int
    nb: int
    kappa_max: float
    src_zx: np.ndarray  # (ns, 2) int32
    rec_zx: np.ndarray  # (nr, 2) int32
    wavelet: np.ndarray  # (nt,) float64
    ckpt_every: int = 50
    inv_noise_var: float = 1.0
    f0: float = 10.0
    meta: dict = field(default_factory=dict)

    @property
    def ns(self) -> int:
        return int(self.src_zx.shape[0])

    @property
    def nr(self) -> int:
        return int(self.rec_zx.shape[0])

    def with_shots(self, idx) -> "Geometry":
        """Same geometry restricted to the listed shots (shots are independent)."""
        idx = np.asarray(idx, dtype=np.int64)
        g = Geometry(**{**self.__dict__})
        g.src_zx = np.ascontiguousarray(self.src_zx[idx])
        g.meta = dict(self.meta)
        return g

    def with_nt(self, nt: int) -> "Geometry":
        g = Geometry(**{**self.__dict__})
        g.nt = int(nt)
        g.wavelet = np.ascontiguousarray(self.wavelet[:nt])
        g.meta = dict(self.meta)
        return g


def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Unit-peak Ricker wavelet sampled at n*dt, delayed by t0 = 1.5/f0."""
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def sponge_strength(cfl: float, nb: int) -> float:
    """Peak damping of the absorbing layer, 3*C*ln(1e3)/(2*nb), capped at
    0.45 so that corner cells (twice the peak) keep a damping below 1."""
    if nb <= 0:
        return 0.0
    return min(3.0 * cfl * math.log(1.0e3) / (2.0 * nb), 0.45)


def surface_shots(nx: int, ns: int, iz: int = 1) -> np.ndarray:
    """ns sources at depth cell iz, centred in ns equal strips of the width."""
    k = np.arange(ns, dtype=np.int64)
    ix = ((2 * k + 1) * nx) // (2 * ns)
    return np.stack([np.full(ns, iz), ix], axis=1).astype(np.int32)


def receiver_line(ix: np.ndarray, iz: int = 1) -> np.ndarray:
    ix = np.asarray(ix, dtype=np.int64)
    return np.stack([np.full(ix.shape[0], iz), ix], axis=1).astype(np.int32)


def make_geometry(nx, nz, *, dx=10.0, nt, ns, rec_ix, f0, v_nominal,
                  cfl=DEFAULT_CFL, nb=20, ckpt_every=50, inv_noise_var=1.0,
                  src_zx=None, rec_iz=1) -> Geometry:
    dt = cfl * dx / v_nominal
    src = surface_shots(nx, ns) if src_zx is None else np.asarray(src_zx, np.int32)
    return Geometry(nx=int(nx), nz=int(nz), dx=float(dx), dt=float(dt), nt=int(nt),
                    nb=int(nb), kappa_max=sponge_strength(cfl, nb),
                    src_zx=np.ascontiguousarray(src, dtype=np.int32),
                    rec_zx=receiver_line(rec_ix, rec_iz),
                    wavelet=ricker(nt, dt, f0), ckpt_every=int(ckpt_every),
                    inv_noise_var=float(inv_noise_var), f0=float(f0),
                    meta={"v_nominal": v_nominal, "cfl": cfl})


def smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing (edge-replicating) over the last two axes."""
    a = np.asarray(a, dtype=np.float64)
    sig = (0,) * (a.ndim - 2) + (sigma, sigma)
    return gaussian_filter(a, sigma=sig, mode="nearest")


# --------------------------------------------------------------------------
# Models
# --------------------------------------------------------------------------

def gaussian_anomaly_model(nx=128, nz=128, dx=10.0, seed=0, background=2000.0,
                           amps=(300.0, -300.0), width=80.0, min_sep=240.0):
    """Background velocity plus seeded Gaussian anomalies (C1 model)."""
    rng = np.random.default_rng(seed)
    Lx, Lz = nx * dx, nz * dx
    if len(amps) > 1 and min_sep >= math.hypot(0.4 * Lz, 0.4 * Lx):
        raise ValueError(f"anomaly centres in the middle 40 % of a {Lz:g} x {Lx:g} m model "
                         f"cannot be {min_sep:g} m apart")
    while True:
        cz = rng.uniform(0.3, 0.7, size=len(amps)) * Lz
        cx = rng.uniform(0.3, 0.7, size=len(amps)) * Lx
        ok = True
        for i in range(len(amps)):
            for j in range(i + 1, len(amps)):
                if math.hypot(cz[i] - cz[j], cx[i] - cx[j]) < min_sep:
                    ok = False
        if ok:
            break
    z = (np.arange(nz) * dx)[:, None]
    x = (np.arange(nx) * dx)[None, :]
    m = np.full((nz, nx), background, dtype=np.float64)
    for a, zc, xc in zip(amps, cz, cx):
        m += a * np.exp(-((z - zc) ** 2 + (x - xc) ** 2) / (2.0 * width ** 2))
    return m


def layered_faulted_model(nx=921, nz=301, dx=10.0, seed=0, n_layers=20,
                          water_depth=300.0, v_water=1500.0, v_top=1600.0,
                          v_bottom=5500.0, n_faults=3):
    """Seeded dipping layers cut by normal faults below a water layer.

    Interface depths are sorted uniform in (water_depth, depth of the grid),
    dips U(-8, 8) degrees about the centre column; layer velocities increase
    from v_top to v_bottom with U(-150, 150) jitter; faults have dip
    U(55, 70) degrees and throw U(50, 200) m (hanging wall down).
    """
    rng = np.random.default_rng(seed)
    Lx, Lz = nx * dx, nz * dx
    xc = 0.5 * Lx
    depths = np.sort(rng.uniform(water_depth, Lz, size=n_layers))
    dips = np.deg2rad(rng.uniform(-8.0, 8.0, size=n_layers))
    vel = np.linspace(v_top, v_bottom, n_layers + 1) + rng.uniform(-150.0, 150.0, n_layers + 1)
    vel = np.clip(np.maximum.accumulate(vel), v_water, v_bottom)
    fx = rng.uniform(0.163 * Lx, 0.837 * Lx, size=n_faults)
    fdip = np.deg2rad(rng.uniform(55.0, 70.0, size=n_faults))
    fthrow = rng.uniform(50.0, 200.0, size=n_faults)
    fside = rng.choice([-1.0, 1.0], size=n_faults)

    z = (np.arange(nz) * dx)[:, None] * np.ones((1, nx))
    x = np.ones((nz, 1)) * (np.arange(nx) * dx)[None, :]
    zs = z.copy()
    for k in range(n_faults):
        # plane through (fx, water_depth); hanging wall on the side it dips to
        xf = fx[k] + fside[k] * (z - water_depth) / math.tan(fdip[k])
        hanging = (fside[k] * (x - xf) > 0) & (z >= water_depth)
        zs = np.where(hanging, zs - fthrow[k], zs)
    idx = np.zeros((nz, nx), dtype=np.int64)
    for k in range(n_layers):
        iface = depths[k] + math.tan(dips[k]) * (x - xc)
        idx += (zs >= iface).astype(np.int64)
    m = vel[idx]
    m[z < water_depth] = v_water
    return m


def smoothed_start(m_true: np.ndarray, sigma: float, water_rows: int = 0,
                   v_water: float = 1500.0) -> np.ndarray:
    """Evaluation model: Gaussian-smoothed truth with the water rows kept."""
    m = smooth(m_true, sigma)
    if water_rows > 0:
        m[:water_rows] = v_water
    return m


# --------------------------------------------------------------------------
# Perturbation / probe vectors
# --------------------------------------------------------------------------

def smooth_random(shape, seed, sigma=5.0) -> np.ndarray:
    """N(0,1) field smoothed by a Gaussian of sigma cells."""
    rng = np.random.default_rng(seed)
    return smooth(rng.standard_normal(shape), sigma)


def smooth_random_batch(nz, nx, seeds, sigma=5.0) -> np.ndarray:
    return np.stack([smooth_random((nz, nx), s, sigma) for s in seeds])


def impulse_combs(nz, nx, count=64, spacing=40, seed=100) -> np.ndarray:
    """count comb probes: unit deltas every `spacing` cells, offsets drawn
    without replacement from [0, spacing)^2."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(spacing * spacing, size=count, replace=False)
    out = np.zeros((count, nz, nx), dtype=np.float64)
    for p, f in enumerate(flat):
        oz, ox = divmod(int(f), spacing)
        out[p, oz::spacing, ox::spacing] = 1.0
    return out


@dataclass(frozen=True)
class PsfGrid:
    """Sample points of the point-spread-function method (Section 3.2) on a
    model grid of nz x nx cells: centres at rows oz + p*sz (p < nzc) and
    columns ox + q*sx (q < nxc), PSF k = p*nxc + q, each PSF kept on the
    window of half-width ``half`` cells around its centre.  The probing
    vectors are ``stride``^2 combs; comb (p % stride)*stride + q % stride holds
    the deltas of every centre with those residues, so deltas of one comb are
    stride*sz rows and stride*sx columns apart."""

    nz: int
    nx: int
    oz: int
    ox: int
    sz: int
    sx: int
    nzc: int
    nxc: int
    half: int
    stride: int = 2

    @property
    def r(self) -> int:
        return self.nzc * self.nxc

    @property
    def width(self) -> int:
        return 2 * self.half + 1

    @property
    def ncombs(self) -> int:
        return self.stride * self.stride

    def centres(self) -> np.ndarray:
        """(r, 2) int array of (iz, ix)."""
        p, q = np.meshgrid(np.arange(self.nzc), np.arange(self.nxc), indexing="ij")
        return np.stack([self.oz + p.ravel() * self.sz, self.ox + q.ravel() * self.sx], axis=1)


def psf_grid(nz, nx, spacing=32, half=None, stride=2) -> PsfGrid:
    """Centres every `spacing` cells, the first half a spacing in from the
    edge, as many as fit; PSF windows as wide as the comb spacing allows
    (2*half + 1 <= stride*spacing, so windows of one comb never overlap)."""
    o = spacing // 2
    nzc = (nz - 1 - o) // spacing + 1
    nxc = (nx - 1 - o) // spacing + 1
    if half is None:
        half = (stride * spacing - 1) // 2
    return PsfGrid(nz, nx, o, o, spacing, spacing, nzc, nxc, half, stride)


def psf_combs(g: PsfGrid) -> np.ndarray:
    """The g.ncombs probing vectors: unit deltas at the centres of each comb."""
    out = np.zeros((g.ncombs, g.nz, g.nx), dtype=np.float64)
    for k, (iz, ix) in enumerate(g.centres()):
        p, q = divmod(k, g.nxc)
        out[(p % g.stride) * g.stride + q % g.stride, iz, ix] = 1.0
    return out


@dataclass(frozen=True)
class Prior:
    """Matern prior precision R = (delta I - gamma Lap_h)^2 on an nz x nx
    model grid of spacing h (Section 2; alpha = 2), Lap_h the 5-point
    Laplacian with mirrored (zero-flux) edges."""

    nz: int
    nx: int
    h: float
    delta: float
    gamma: float


def matern_prior(nz, nx, h, corr_length, std) -> Prior:
    """delta and gamma from a correlation length and a pointwise standard
    deviation, by the continuous Matern relations for alpha = 2 in 2-D
    (smoothness nu = 1): kappa = sqrt(8 nu) / rho, sigma^2 =
    1 / (4 pi kappa^2 gamma^2), delta = kappa^2 gamma."""
    kappa = math.sqrt(8.0) / corr_length
    gamma = 1.0 / (std * kappa * math.sqrt(4.0 * math.pi))
    return Prior(nz, nx, h, kappa * kappa * gamma, gamma)


@dataclass(frozen=True)
class SymbolGrid:
    """Periodic FFT grid of mz x mx cells of spacing h whose first nz rows and
    nx columns hold the model grid (the rest is zero padding), and the
    sampling of the symbol columns: r equally spaced directions on the circle
    of radius rho0 (angular wavenumber, rad per unit length)."""

    nz: int
    nx: int
    mz: int
    mx: int
    h: float
    r: int = 8
    rho0: float = 0.0


def fft_size(n: int) -> int:
    """Smallest m >= n whose prime factors are 2, 3 and 5."""
    m = max(int(n), 1)
    while True:
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


def symbol_grid(nz, nx, h, pad, r=8, rho0=0.0) -> SymbolGrid:
    """FFT grid with at least `pad` cells of zero padding after the model in
    each direction (pad >= the half width of a PSF window keeps circular
    correlations with such windows free of wrap-around)."""
    return SymbolGrid(nz, nx, fft_size(nz + pad), fft_size(nx + pad), float(h), int(r),
                      float(rho0))


def probe_radius(f_max: float, c_max: float) -> float:
    """Angular wavenumber 2 pi f_max / c_max of the shortest wavelength the
    band reaches at the highest velocity."""
    return 2.0 * math.pi * f_max / c_max


def gaussian_probes(nz, nx, count, seed) -> np.ndarray:
    """count N(0, 1) fields: the random test matrix of a randomized method."""
    return np.random.default_rng(seed).standard_normal((count, nz, nx))


def rademacher_smoothed(nz, nx, seeds, sigma=5.0) -> np.ndarray:
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        out.append(smooth(rng.choice([-1.0, 1.0], size=(nz, nx)), sigma))
    return np.stack(out)


def residual_noise(shape, seed) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def config_small():
    """128x128 model, 4 surface shots, 32 receivers, Ricker 10 Hz, 500 steps."""
    m_true = gaussian_anomaly_model(seed=0)
    m_eval = smoothed_start(m_true, 5.0)
    g = make_geometry(128, 128, nt=500, ns=4, rec_ix=2 + 4 * np.arange(32),
                      f0=10.0, v_nominal=2300.0)
    return g, m_true, m_eval


def config_layered(nx=921, nz=301, ns=64, nt=4000, nr=None, seed=0, ckpt_every=50):
    """Layered-faulted model, full-width receiver line every 2 cells."""
    m_true = layered_faulted_model(nx, nz, seed=seed)
    water_rows = int(round(300.0 / 10.0))
    m_eval = smoothed_start(m_true, 10.0, water_rows=water_rows)
    if nr is None:
        nr = (nx + 1) // 2
    g = make_geometry(nx, nz, nt=nt, ns=ns, rec_ix=2 * np.arange(nr), f0=8.0,
                      v_nominal=5500.0, ckpt_every=ckpt_every)
    return g, m_true, m_eval
