"""Seeded synthetic inputs: density grids, source lists and scene descriptions.

This module is shared by the GPU library's tests/bench and by the CPU oracle, so it
holds no arithmetic of the method itself (no Gladstone-Dale, no ray equation, no
optics): only the scene geometry and the seeded generators of the density field and of
the particle / dot positions.

Scenes follow the paper's BOS set-up (Table 1 of section 4: Z_D = 0.25 m, Z_A = 0.75 m,
f = 105 mm at f/11, 10 um pixels, density scaled by 1.225 kg/m^3) and its Tomo-PIV sizing
(section 2: 1e5 particles in a 300 cm^3 volume, 1e4 rays per particle).  The paper's DNS
field (section 4, JHU turbulence database) is not available; a seeded random-phase field
with a k^-5/3 spectrum stands in for it.

Geometry convention: the optical axis is +z, light travels towards +z; sources sit at
small z, then the density box, then the lens front vertex at ``z_lens``, then the sensor.
x and y are centred on the axis.  All lengths are metres.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# Gladstone-Dale constant for air, 0.226 cm^3/g (section 3.2), in m^3/kg.
K_AIR = 2.26e-4


@dataclass(frozen=True)
class Scene:
    """Everything one image needs: grid, field recipe, sources, optics, sensor, step."""

    name: str
    # density grid: node counts, position of node (0,0,0), node spacing
    nx: int
    ny: int
    nz: int
    origin: tuple
    spacing: tuple
    field: str  # 'uniform' | 'bump' | 'turbulence' | 'slice' | 'shock' | 'linear'
    field_params: dict = dataclasses.field(default_factory=dict)
    K: float = K_AIR
    rho_inf: float = 1.2
    # sources
    source_kind: str = "dots"  # 'dots' (plane z = const) | 'particles' (inside a box)
    n_src: int = 1000
    src_region: tuple = ((-0.024, 0.024), (-0.024, 0.024), (0.0, 0.0))
    src_seed: int = 1
    rays_per_src: int = 100
    ray_seed: int = 1
    # optics: thick symmetric biconvex lens, aperture stop at the front vertex plane
    z_lens: float = 0.5
    focal_length: float = 0.05
    f_number: float = 8.0
    n_glass: float = 1.5
    thickness: float = 0.0  # <= 0 means 0.1 * focal_length
    clear_radius: float = 0.0  # <= 0 means 1.5 * aperture radius
    z_focus: float = 0.0  # object plane imaged sharply when the sensor is auto-placed
    # sensor
    width: int = 256
    height: int = 256
    pitch: float = 20e-6
    z_sensor: float = float("nan")  # NaN: place the sensor at the paraxial image of z_focus
    wavelength: float = 532e-9  # effective green wavelength for white light (section 3.4)
    sigma_px: float = 0.0  # <= 0: diffraction spot from eq. 8
    dtau_with_pi: bool = False
    # integration
    ds: float = 1e-4

    @property
    def n_rays(self) -> int:
        return int(self.n_src) * int(self.rays_per_src)

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)

    def box_max(self):
        return tuple(o + (n - 1) * h for o, n, h in
                     zip(self.origin, (self.nx, self.ny, self.nz), self.spacing))


def _centred_box(n, extent, zc):
    """origin/spacing of an n-node grid spanning ``extent`` (x, y, z), centred on the axis
    with its mid-plane at z = zc."""
    sp = tuple(e / (k - 1) for e, k in zip(extent, n))
    org = (-extent[0] / 2, -extent[1] / 2, zc - extent[2] / 2)
    return org, sp


def tiny_bos() -> Scene:
    """Plain tracer, tiny BOS image: 32^3 Gaussian bump in a 5 cm cube, 1000 dots x 100 rays,
    f = 50 mm f/8, 256^2 sensor of 20 um pixels, ds = 0.1 mm."""
    org, sp = _centred_box((32, 32, 32), (0.05, 0.05, 0.05), 0.125)
    return Scene(
        name="tiny_bos_32", nx=32, ny=32, nz=32, origin=org, spacing=sp,
        field="bump",
        field_params=dict(rho0=1.2, amp=0.1, sigma=0.01, centre=(0.0, 0.0, 0.125)),
        rho_inf=1.2, source_kind="dots", n_src=1000,
        src_region=((-0.024, 0.024), (-0.024, 0.024), (0.0, 0.0)), src_seed=1,
        rays_per_src=100, ray_seed=1,
        z_lens=0.5, focal_length=0.05, f_number=8.0, z_focus=0.0,
        width=256, height=256, pitch=20e-6, ds=1e-4)


def turbulence_bos(n: int = 128, seed: int = 2, n_src: int = 50_000,
                   rays_per_src: int = 1000) -> Scene:
    """BOS through a synthetic buoyancy-driven-turbulence stand-in: n^3 random-phase field
    with a k^-5/3 spectrum, density ratio 1.05, periodic 2*pi box scaled to 10 cm, 50 000 dots
    x 1000 rays, Table 1 geometry (Z_D 0.25 m, Z_A 0.75 m), f = 105 mm f/11, 1024^2 x 10 um."""
    h = 0.1 / n
    ext = (n - 1) * h
    org, sp = _centred_box((n, n, n), (ext, ext, ext), 0.25)
    return Scene(
        name=f"turbulence_bos_{n}", nx=n, ny=n, nz=n, origin=org, spacing=sp,
        field="turbulence", field_params=dict(rho0=1.225, ratio=1.05, kmax=16, seed=seed),
        rho_inf=1.225, source_kind="dots", n_src=n_src,
        src_region=((-0.045, 0.045), (-0.045, 0.045), (0.0, 0.0)), src_seed=20,
        rays_per_src=rays_per_src, ray_seed=2,
        z_lens=1.0, focal_length=0.105, f_number=11.0, z_focus=0.0,
        width=1024, height=1024, pitch=10e-6, ds=1e-4)


def tomo_piv_shock(n: int = 512, n_src: int = 100_000, rays_per_src: int = 10_000) -> Scene:
    """Tomo-PIV scale: n^3 grid over 10 x 10 x 3 cm (300 cm^3) holding a normal shock, a tanh
    density step 1.2 -> 3.0 kg/m^3 over about 0.2 mm, 1e5 particles x 1e4 rays, f = 105 mm f/11
    focused on the mid-plane (magnification about 0.205), 2048^2 x 10 um sensor, 16-bit output."""
    org, sp = _centred_box((n, n, n), (0.1, 0.1, 0.03), 0.0)
    return Scene(
        name=f"tomo_piv_shock_{n}", nx=n, ny=n, nz=n, origin=org, spacing=sp,
        field="shock", field_params=dict(rho1=1.2, rho2=3.0, delta=1e-4, x_s=0.0),
        rho_inf=1.2, source_kind="particles", n_src=n_src,
        src_region=((-0.05, 0.05), (-0.05, 0.05), (-0.015, 0.015)), src_seed=3,
        rays_per_src=rays_per_src, ray_seed=3,
        z_lens=0.614, focal_length=0.105, f_number=11.0, z_focus=0.0,
        width=2048, height=2048, pitch=10e-6, ds=1e-4)


def surrogate_turbulence():
    """Surrogate workload: the turbulence BOS scene on a 256^3 grid (field seed 5, node spacing
    0.39 mm), ds = 0.1 mm.  Returns (evaluation, training, validation) scenes that differ only in
    their dots: 1e6 dots x 1000 rays for evaluation (1e9 rays, ray seed 51), 1e4 x 1000 for
    training (1e7 rays, seed 50), 1e5 x 10 for validation (1e6 rays, seed 52; many dots with few
    rays each, so that every tile of the entry face receives validation rays)."""
    ev = turbulence_bos(n=256, seed=5, n_src=1_000_000, rays_per_src=1000).replace(
        name="surrogate_turbulence_256", src_seed=510, ray_seed=51)
    tr = ev.replace(n_src=10_000, src_seed=500, ray_seed=50)
    va = ev.replace(n_src=100_000, rays_per_src=10, src_seed=520, ray_seed=52)
    return ev, tr, va


def bos_slice(n: int = 257, seed: int = 6, n_src: int = 5200, rays_per_src: int = 1000) -> Scene:
    """The BOS experiment of section 4 (Fig. 3, Table 1) on a synthetic stand-in for its DNS
    slice: one 2-D random-phase slice (k^-5/3 energy spectrum, density ratio 1.05, scaled by
    1.225 kg/m^3) stacked along z, so that the density has no z gradient.  Box 32 x 32 x 10 mm
    (n x n x nz nodes, 0.125 mm spacing at n = 257), centre at Z_D = 0.25 m from the dot plane
    z = 0, lens front vertex Z_A = 0.75 m beyond the centre; f = 105 mm at f/11 focused on the
    dots (magnification about 0.117); 512^2 sensor of 10 um pixels; 20 dots per 32 x 32 pixels
    over the 44 x 44 mm of the dot plane the sensor sees (5200 dots), 1000 rays each."""
    h = 0.032 / (n - 1)
    nz = int(round(0.010 / h)) + 1
    org = (-0.016, -0.016, 0.25 - 0.5 * (nz - 1) * h)
    return Scene(
        name=f"bos_slice_{n}", nx=n, ny=n, nz=nz, origin=org, spacing=(h, h, h),
        field="slice", field_params=dict(rho0=1.225, ratio=1.05, kmax=16, seed=seed),
        rho_inf=1.225, source_kind="dots", n_src=n_src,
        src_region=((-0.022, 0.022), (-0.022, 0.022), (0.0, 0.0)), src_seed=60,
        rays_per_src=rays_per_src, ray_seed=61,
        z_lens=1.0, focal_length=0.105, f_number=11.0, z_focus=0.0,
        width=512, height=512, pitch=10e-6, ds=1e-4)


def map_grid(scene: Scene, nodes: int = 64, half_width: float = 0.020):
    """Regular grid of the displacement maps on the dot plane z = src_region[2][0]: nodes x nodes
    points spanning [-half_width, half_width]^2.  Returns (x0, y0, dx, dy, nx, ny, z_dots)."""
    d = 2.0 * half_width / (nodes - 1)
    return (-half_width, -half_width, d, d, nodes, nodes, float(scene.src_region[2][0]))


def synthetic_source_sums(n: int, seed: int, width: int, height: int, max_hits: int = 1000):
    """Two seeded arrays of per-source hit sums in the layout of the per-source sum records
    (int64 [n][4] = sum_x, sum_y, hits, 0; sums in units of 2^-24 pixel), as a render with and
    one without a field would leave them: hit counts in [0, max_hits] (about 3% zero), mean hits
    uniform on the sensor, the second set shifted by up to 2 pixels.  Sums stay below 2^53."""
    rng = np.random.default_rng(seed)
    out = []
    hits = rng.integers(0, max_hits + 1, size=n)
    hits[rng.random(n) < 0.03] = 0
    mx = rng.uniform(0, width, n)
    my = rng.uniform(0, height, n)
    for k in range(2):
        if k:
            hits = np.where(rng.random(n) < 0.02, 0, hits)
            mx = mx + rng.uniform(-2, 2, n)
            my = my + rng.uniform(-2, 2, n)
        a = np.zeros((n, 4), dtype=np.int64)
        a[:, 0] = np.rint(mx * hits * 2.0 ** 24).astype(np.int64)
        a[:, 1] = np.rint(my * hits * 2.0 ** 24).astype(np.int64)
        a[:, 2] = hits
        out.append(a)
    return out[0], out[1]


def velocity_field(kind: str, n: int = 33, region=((-0.05, 0.05), (-0.05, 0.05), (-0.015, 0.015)),
                   **p):
    """A prescribed velocity field sampled on an n^3 grid over ``region`` (PIV frame pairs: the
    second frame's particles are moved by it).  Returns (vel float32 [n][n][n][3] as [iz][iy][ix]
    of (u, v, w) in m/s, origin, spacing).  Kinds:
      'uniform'  u = p['u'] (3-vector);
      'shear'    u = (gamma * y, 0, 0);
      'rotation' solid-body rotation about the z axis through p['centre'] at p['omega'] rad/s;
      'vortex'   Lamb-Oseen vortex about the z axis through p['centre'], circulation p['gamma']
                 (m^2/s), core radius p['rc'] (m): u_theta = gamma / (2 pi r) (1 - exp(-r^2/rc^2)),
                 plus a uniform stream p.get('u', 0)."""
    (x0, x1), (y0, y1), (z0, z1) = region
    org = (x0, y0, z0)
    sp = ((x1 - x0) / (n - 1), (y1 - y0) / (n - 1), (z1 - z0) / (n - 1))
    x = x0 + sp[0] * np.arange(n)
    y = y0 + sp[1] * np.arange(n)
    X = np.broadcast_to(x[None, None, :], (n, n, n))
    Y = np.broadcast_to(y[None, :, None], (n, n, n))
    vel = np.zeros((n, n, n, 3))
    if kind == "uniform":
        vel[...] = np.asarray(p["u"], dtype=np.float64)
    elif kind == "shear":
        vel[..., 0] = p["gamma"] * Y
    elif kind == "rotation":
        cx, cy = p.get("centre", (0.0, 0.0))
        vel[..., 0] = -p["omega"] * (Y - cy)
        vel[..., 1] = p["omega"] * (X - cx)
    elif kind == "vortex":
        cx, cy = p.get("centre", (0.0, 0.0))
        dx, dy = X - cx, Y - cy
        r2 = dx * dx + dy * dy
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(r2 > 0, p["gamma"] / (2 * np.pi * r2) * (1 - np.exp(-r2 / p["rc"] ** 2)),
                         p["gamma"] / (2 * np.pi * p["rc"] ** 2))
        vel[..., 0] = -f * dy
        vel[..., 1] = f * dx
        vel[...] += np.asarray(p.get("u", (0.0, 0.0, 0.0)), dtype=np.float64)
    else:
        raise ValueError(f"unknown velocity field {kind!r}")
    return np.ascontiguousarray(vel, dtype=np.float32), org, sp


def piv_pair_flow(n: int = 65):
    """Velocity of the PIV pair workload: a Lamb-Oseen vortex about the optical axis
    (circulation 0.05 m^2/s, core radius 1 cm) in a 0.2 m/s stream along x, on an n^3 grid over
    the Tomo-PIV particle volume; frame interval 0.5 ms (particle images move up to ~7 pixels).
    Returns (vel, origin, spacing, dt)."""
    vel, org, sp = velocity_field("vortex", n, gamma=0.05, rc=0.01, u=(0.2, 0.0, 0.0))
    return vel, org, sp, 5e-4


def batch_scenes(n_images: int = 64, seed_base: int = 4000):
    """Many images of uneven sizes: particle counts log-uniform in [1e3, 1e5], rays per particle
    log-uniform in [500, 1e4], grids 64^3 / 128^3 / 256^3 holding a Gaussian bump or a
    turbulence field, sensors 512^2 .. 2048^2.  Particles fill a 10 cm cube centred at z = 0,
    imaged by the f = 105 mm f/11 lens focused on z = 0."""
    out = []
    for i in range(n_images):
        rng = np.random.default_rng(seed_base + i)
        n_p = int(round(10 ** rng.uniform(3, 5)))
        rpp = int(round(10 ** rng.uniform(math.log10(500), 4)))
        n = int(rng.choice([64, 128, 256]))
        kind = str(rng.choice(["bump", "turbulence"]))
        w = int(rng.choice([512, 1024, 2048]))
        org, sp = _centred_box((n, n, n), (0.1, 0.1, 0.1), 0.0)
        if kind == "bump":
            c = tuple(float(v) for v in rng.uniform(-0.025, 0.025, size=3))
            fp = dict(rho0=1.2, amp=float(rng.uniform(0.05, 0.2)),
                      sigma=float(rng.uniform(0.005, 0.02)), centre=c)
        else:
            fp = dict(rho0=1.2, ratio=1.05, kmax=16, seed=seed_base + i)
        out.append(Scene(
            name=f"batch_{i:02d}", nx=n, ny=n, nz=n, origin=org, spacing=sp, field=kind,
            field_params=fp, rho_inf=1.2, source_kind="particles", n_src=n_p,
            src_region=((-0.05, 0.05), (-0.05, 0.05), (-0.05, 0.05)), src_seed=seed_base + i,
            rays_per_src=rpp, ray_seed=seed_base + i,
            z_lens=0.614, focal_length=0.105, f_number=11.0, z_focus=0.0,
            width=w, height=w, pitch=10e-6 * 2048 / w, ds=1e-4))
    return out


# ----------------------------------------------------------------------------- fields

def node_axes(scene: Scene):
    """Node coordinates along x, y, z (float64)."""
    return tuple(o + h * np.arange(k, dtype=np.float64)
                 for o, h, k in zip(scene.origin, scene.spacing, (scene.nx, scene.ny, scene.nz)))


def turbulence_psi(n: int, kmax: int, seed: int) -> np.ndarray:
    """Random-phase field psi(x) = sum_{k in Z^3, 1 <= |k| <= kmax} |k|^(-11/6) cos(k.x + phi_k)
    sampled at x = 2*pi*i/n on [0, 2*pi)^3 (so the 3-D energy spectrum goes as k^-5/3).
    Phases phi_k ~ U[0, 2*pi) are drawn from ``seed`` in lexicographic (kx, ky, kz) order.
    Returned as [iz, iy, ix], float64.  Built with one inverse FFT."""
    if 2 * kmax >= n:
        raise ValueError("kmax must be below n/2")
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(r, r, r, indexing="ij")
    kk = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    m = (kk >= 1) & (kk <= kmax)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=int(m.sum()))
    amps = kk[m] ** (-11.0 / 6.0)
    F = np.zeros((n, n, n), dtype=np.complex128)
    F[KZ[m] % n, KY[m] % n, KX[m] % n] = amps * np.exp(1j * phases)
    psi = np.fft.ifftn(F).real * float(n) ** 3
    return psi


def turbulence_psi2(n: int, kmax: int, seed: int) -> np.ndarray:
    """2-D random-phase field psi(x, y) = sum_{k in Z^2, 1 <= |k| <= kmax} |k|^(-4/3)
    cos(k.x + phi_k) at x = 2*pi*i/n on [0, 2*pi)^2 (energy spectrum k^-5/3 in the plane),
    phases from ``seed`` in lexicographic (kx, ky) order.  Returned as [iy, ix], float64."""
    if 2 * kmax >= n:
        raise ValueError("kmax must be below n/2")
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(r, r, indexing="ij")
    kk = np.sqrt(KX * KX + KY * KY)
    m = (kk >= 1) & (kk <= kmax)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=int(m.sum()))
    amps = kk[m] ** (-4.0 / 3.0)
    F = np.zeros((n, n), dtype=np.complex128)
    F[KY[m] % n, KX[m] % n] = amps * np.exp(1j * phases)
    return np.fft.ifft2(F).real * float(n) ** 2


def density(scene: Scene) -> np.ndarray:
    """Density rho [kg/m^3] at the grid nodes, float32, C-contiguous [nz][ny][nx]."""
    fp = scene.field_params
    x, y, z = node_axes(scene)
    shape = (scene.nz, scene.ny, scene.nx)
    if scene.field == "uniform":
        rho = np.full(shape, fp.get("rho0", scene.rho_inf), dtype=np.float64)
    elif scene.field == "bump":
        cx, cy, cz = fp["centre"]
        s2 = 2.0 * fp["sigma"] ** 2
        gx = np.exp(-(x - cx) ** 2 / s2)
        gy = np.exp(-(y - cy) ** 2 / s2)
        gz = np.exp(-(z - cz) ** 2 / s2)
        rho = fp["rho0"] * (1.0 + fp["amp"] * gz[:, None, None] * gy[None, :, None]
                            * gx[None, None, :])
    elif scene.field == "turbulence":
        if not (scene.nx == scene.ny == scene.nz):
            raise ValueError("turbulence field needs a cubic grid")
        psi = turbulence_psi(scene.nx, fp.get("kmax", 16), fp["seed"])
        psi_hat = (psi - psi.min()) / (psi.max() - psi.min())
        rho = fp["rho0"] * (1.0 + (fp["ratio"] - 1.0) * psi_hat)
    elif scene.field == "slice":
        # one x-y slice stacked along z: the density has no z gradient
        if scene.nx != scene.ny:
            raise ValueError("slice field needs nx == ny")
        psi = turbulence_psi2(scene.nx, fp.get("kmax", 16), fp["seed"])
        psi_hat = (psi - psi.min()) / (psi.max() - psi.min())
        sl = fp["rho0"] * (1.0 + (fp["ratio"] - 1.0) * psi_hat)
        rho = np.broadcast_to(sl[None, :, :], shape)
    elif scene.field == "shock":
        r1, r2 = fp["rho1"], fp["rho2"]
        prof = r1 + 0.5 * (r2 - r1) * (1.0 + np.tanh((x - fp["x_s"]) / fp["delta"]))
        rho = np.broadcast_to(prof[None, None, :], shape)
    elif scene.field == "linear":
        # rho = rho0 + g . (X - X0): exercises exact-gradient cases
        g = fp["grad"]
        x0 = fp.get("x0", (0.0, 0.0, 0.0))
        rho = (fp["rho0"] + g[0] * (x - x0[0])[None, None, :] + g[1] * (y - x0[1])[None, :, None]
               + g[2] * (z - x0[2])[:, None, None])
        rho = np.broadcast_to(rho, shape)
    else:
        raise ValueError(f"unknown field kind {scene.field!r}")
    return np.ascontiguousarray(rho, dtype=np.float32)


def sources(scene: Scene) -> np.ndarray:
    """Source list float32 [n_src][4] = (x, y, z, weight); weight 1.  Dots are uniform on the
    rectangle ``src_region`` at the plane z = src_region[2][0]; particles are uniform in the
    box ``src_region``.  Seeded by ``src_seed``."""
    rng = np.random.default_rng(scene.src_seed)
    (x0, x1), (y0, y1), (z0, z1) = scene.src_region
    n = int(scene.n_src)
    out = np.empty((n, 4), dtype=np.float64)
    out[:, 0] = rng.uniform(x0, x1, n)
    out[:, 1] = rng.uniform(y0, y1, n)
    out[:, 2] = z0 if scene.source_kind == "dots" else rng.uniform(z0, z1, n)
    out[:, 3] = 1.0
    return out.astype(np.float32)


SCENES = {
    "tiny_bos": tiny_bos,
    "turbulence_bos": turbulence_bos,
    "tomo_piv_shock": tomo_piv_shock,
    "bos_slice": bos_slice,
}
