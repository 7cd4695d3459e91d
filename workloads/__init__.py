"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds *inputs only*: wall-normal face coordinates, triangulated
surfaces, the host-side kinematic coefficients of each body (every
transcendental is evaluated here, on the host) and the initial velocity
fields.  It holds none of the method's arithmetic: no tagging, no forcing, no
differential operator, no solver.  Both the CPU oracle and the HIP path consume
the arrays produced here, so the two sides see bit-identical inputs without
sharing any code.

Shapes follow the paper's workloads (a periodic channel, x1/x2 periodic and
uniform, x3 stretched, Sec. 2; plates of the heaving/pitching test, Sec. 4.4;
spheres of the settling tests, Sec. 4.5; closed deforming membranes of the
bubble test, Sec. 4.7).  The paper evaluates on no public dataset; these
seeded generators stand in for its setups, whose data is not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "uniform_faces", "tanh_faces", "icosphere", "plate_mesh",
    "rigid_coef", "sphere_translation", "plate_heave_pitch",
    "deform_vertex_data", "deform_coef", "splitmix64_uniform", "splitmix64_uniform_torch",
    "initial_velocity", "initial_velocity_torch", "Workload", "config", "CONFIG_NAMES", "batch_sim", "batch",
]

# --------------------------------------------------------------------------
# wall-normal grids (the caller-supplied face coordinates y_f[0..ny])
# --------------------------------------------------------------------------

def uniform_faces(ny: int, y0: float = -1.0, y1: float = 1.0) -> np.ndarray:
    """ny+1 uniformly spaced faces on [y0, y1] (end points exact)."""
    j = np.arange(ny + 1, dtype=np.float64)
    yf = y0 + (y1 - y0) * j / ny
    yf[0], yf[-1] = y0, y1
    return yf


def tanh_faces(ny: int, beta: float = 2.0) -> np.ndarray:
    """ny+1 faces on [-1, 1] clustered at both walls:
    y_f[j] = tanh(beta*(2j/ny - 1)) / tanh(beta).  For even ny the middle face
    is exactly 0."""
    j = np.arange(ny + 1, dtype=np.float64)
    yf = np.tanh(beta * (2.0 * j / ny - 1.0)) / math.tanh(beta)
    yf[0], yf[-1] = -1.0, 1.0
    if ny % 2 == 0:
        yf[ny // 2] = 0.0
    return yf

# --------------------------------------------------------------------------
# triangulated surfaces
# --------------------------------------------------------------------------

def icosphere(level: int):
    """Unit icosphere: 20*4**level triangles, outward counter-clockwise.
    Returns (verts f64[nv,3], tris i32[nt,3])."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1.0 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts, dtype=np.float64)
    F = np.array(faces, dtype=np.int32)
    # orient outward: (B-A)x(C-A) points away from the centre
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", n, V[F].mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def plate_mesh(chord: float, span: float, nq_x: int, nq_z: int):
    """Zero-thickness flat plate in the x-z plane (y = 0), centred at the
    origin: chord along x, span along z, nq_x*nq_z quads split by a fixed
    diagonal into 2*nq_x*nq_z triangles.  Returns (verts, tris)."""
    xs = -0.5 * chord + chord * np.arange(nq_x + 1, dtype=np.float64) / nq_x
    zs = -0.5 * span + span * np.arange(nq_z + 1, dtype=np.float64) / nq_z
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    V = np.stack([X.ravel(), np.zeros(X.size), Z.ravel()], axis=1)
    tris = []
    for a in range(nq_x):
        for b in range(nq_z):
            v00 = a * (nq_z + 1) + b
            v10 = (a + 1) * (nq_z + 1) + b
            v01 = v00 + 1
            v11 = v10 + 1
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    return V, np.array(tris, dtype=np.int32)

# --------------------------------------------------------------------------
# host-side kinematics: coefficients only (every sin/cos is taken here)
# --------------------------------------------------------------------------

def rigid_coef(c, R, cdot, omega) -> np.ndarray:
    """Pack a rigid motion X = c + R X0, U = cdot + omega x (X - c) into the
    18-double coefficient vector [c(3), R(9, row-major), cdot(3), omega(3)]."""
    out = np.empty(18, dtype=np.float64)
    out[0:3] = c
    out[3:12] = np.asarray(R, dtype=np.float64).reshape(9)
    out[12:15] = cdot
    out[15:18] = omega
    return out


def sphere_translation(t: float, c0, U) -> np.ndarray:
    """Rigid translation at constant velocity U from centre c0."""
    c0 = np.asarray(c0, np.float64)
    U = np.asarray(U, np.float64)
    return rigid_coef(c0 + U * t, np.eye(3), U, np.zeros(3))


def plate_heave_pitch(t: float, centre=(math.pi, 0.0, 0.5 * math.pi),
                      heave=0.2, freq=1.0, pitch=math.pi / 12.0) -> np.ndarray:
    """Heaving (along y) and pitching (about z through the centre) plate:
    y_c = heave*sin(2 pi f t), theta = pitch*sin(4 pi f t) (pitch at twice the
    heave frequency, as in the heaving/pitching plate test)."""
    w = 2.0 * math.pi * freq
    th = pitch * math.sin(2.0 * w * t)
    thd = pitch * 2.0 * w * math.cos(2.0 * w * t)
    ct, st = math.cos(th), math.sin(th)
    R = [[ct, -st, 0.0], [st, ct, 0.0], [0.0, 0.0, 1.0]]
    c = (centre[0], centre[1] + heave * math.sin(w * t), centre[2])
    cd = (0.0, heave * w * math.cos(w * t), 0.0)
    return rigid_coef(c, R, cd, (0.0, 0.0, thd))


def deform_vertex_data(unit_verts: np.ndarray, r0: float, amp: float = 0.1):
    """Per-vertex data of the deforming closed body
    r(theta, t) = r0 (1 + amp Y20(theta) sin(4 pi t)), theta from +y:
    returns f64[nv,4] = [direction(3), r0*amp*Y20(theta)]."""
    d = unit_verts / np.linalg.norm(unit_verts, axis=1, keepdims=True)
    ct = d[:, 1]
    y20 = 0.25 * math.sqrt(5.0 / math.pi) * (3.0 * ct * ct - 1.0)
    out = np.empty((len(d), 4), dtype=np.float64)
    out[:, :3] = d
    out[:, 3] = r0 * amp * y20
    return out


def deform_coef(t: float, centre, r0: float, freq: float = 2.0, U=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Scalars of the deforming body at time t: [c(3), r0, s, sdot, cdot(3)]
    with s = sin(2 pi freq t) and the centre c = centre + U t moving at
    cdot = U."""
    w = 2.0 * math.pi * freq
    return np.array([centre[0] + U[0] * t, centre[1] + U[1] * t, centre[2] + U[2] * t, r0,
                     math.sin(w * t), w * math.cos(w * t), U[0], U[1], U[2]], dtype=np.float64)

# --------------------------------------------------------------------------
# initial fields
# --------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64_uniform(seed: int, comp: int, n: int, start: int = 0) -> np.ndarray:
    """xi in [0,1) with 53 random bits: SplitMix64 (Steele, Lea, Flood 2014)
    applied to the counter (seed << 34) | (comp << 32) | index."""
    with np.errstate(over="ignore"):
        idx = np.arange(start, start + n, dtype=np.uint64)
        x = (np.uint64(seed) << np.uint64(34)) | (np.uint64(comp) << np.uint64(32)) | idx
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def splitmix64_uniform_torch(seed: int, comp: int, n: int, device, start: int = 0):
    """The same values as splitmix64_uniform, computed by torch on `device`
    (int64 arithmetic wraps like uint64; logical right shifts are arithmetic
    shifts masked to the low 64-k bits)."""
    import torch

    def srl(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    def c64(v):  # a uint64 constant as the int64 with the same bits
        return v - (1 << 64) if v >= (1 << 63) else v

    idx = torch.arange(start, start + n, dtype=torch.int64, device=device)
    z = idx | ((int(seed) << 34) | (int(comp) << 32))
    z = z + c64(0x9E3779B97F4A7C15)
    z = (z ^ srl(z, 30)) * c64(0xBF58476D1CE4E5B9)
    z = (z ^ srl(z, 27)) * c64(0x94D049BB133111EB)
    z = z ^ srl(z, 31)
    return srl(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def _profile(yn, uc, half, profile):
    if profile is not None:
        return np.asarray(profile(yn), np.float64)
    yh = yn / half
    return uc * (1.0 - yh * yh)


def initial_velocity_torch(nx, ny, nz, y_faces, uc=1.0, amp=0.01, seed=1, half=1.0,
                           device="cpu", profile=None):
    """initial_velocity computed by torch on `device`, plane by plane (the
    same values bit for bit; flat tensors u, v, w)."""
    import torch
    yf = np.asarray(y_faces, np.float64)
    prof = torch.from_numpy(_profile((yf[:-1] + yf[1:]) * 0.5, uc, half, profile)).to(device)
    plane = nx * nz
    u = torch.empty(ny * plane, dtype=torch.float64, device=device)
    v = torch.zeros((ny + 1) * plane, dtype=torch.float64, device=device)
    w = torch.empty(ny * plane, dtype=torch.float64, device=device)
    step = max(1, (1 << 26) // plane)  # planes per chunk
    for j0 in range(0, ny, step):
        j1 = min(ny, j0 + step)
        a, b = j0 * plane, j1 * plane
        xi = splitmix64_uniform_torch(seed, 0, b - a, device, start=a)
        u[a:b] = prof[j0:j1].repeat_interleave(plane) + amp * (2.0 * xi - 1.0)
        w[a:b] = amp * (2.0 * splitmix64_uniform_torch(seed, 2, b - a, device, start=a) - 1.0)
        jv1 = min(j1, ny - 1)
        if jv1 > j0:   # interior v planes j = 1..ny-1, counter index (j-1)*plane + ...
            av, bv = j0 * plane, jv1 * plane
            v[plane + av:plane + bv] = amp * (2.0 * splitmix64_uniform_torch(
                seed, 1, bv - av, device, start=av) - 1.0)
    return u, v, w


def initial_velocity(nx, ny, nz, y_faces, uc=1.0, amp=0.01, seed=1, half=1.0, profile=None):
    """Laminar profile u = uc (1 - (y/half)^2) at the u-node heights (walls at
    y = -half and +half; or profile(y) when given) plus a seeded uniform
    perturbation amp*(2 xi - 1) on every interior u, v, w unknown.  Layout
    [y][z][x]; v has ny+1 planes, the wall planes are 0.  Returns (u, v, w)
    f64 arrays."""
    yf = np.asarray(y_faces, np.float64)
    yn = (yf[:-1] + yf[1:]) * 0.5                     # u-node heights
    n = nx * ny * nz
    u = _profile(yn, uc, half, profile)[:, None, None] * np.ones((ny, nz, nx))
    u += amp * (2.0 * splitmix64_uniform(seed, 0, n).reshape(ny, nz, nx) - 1.0)
    v = np.zeros((ny + 1, nz, nx))
    nv = (ny - 1) * nz * nx
    v[1:ny] = amp * (2.0 * splitmix64_uniform(seed, 1, nv).reshape(ny - 1, nz, nx) - 1.0)
    w = amp * (2.0 * splitmix64_uniform(seed, 2, n).reshape(ny, nz, nx) - 1.0)
    return u, v, w

# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Body:
    kind: str                  # "rigid" or "deform"
    ref: np.ndarray            # rigid: X0 (relative to centre) f64[nv,3];
                               # deform: f64[nv,4] [dir, amplitude]
    tris: np.ndarray           # i32[nt,3]
    coef: object               # callable t -> coefficient vector


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    y_faces: np.ndarray
    re: float
    dt: float
    steps: int
    uc: float
    amp: float
    seed: int
    dpdx: float                # mean pressure gradient dP/dx (driving force -dP/dx)
    bodies: list = field(default_factory=list)
    scheme: str = "rk2"
    half: float = 1.0          # channel half-height (walls at +-half)
    # the initial laminar profile u(y) at the u-node heights (None: the
    # parabola uc (1 - (y/half)^2) of a channel with walls at +-half)
    profile: object = None
    # volume force of the immersed-plane channels of Sec. 4.2 / 4.3
    # ("vortex" / "relax"; None: only the constant driving gradient dpdx)
    vforce: object = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def fields(self):
        return initial_velocity(self.nx, self.ny, self.nz, self.y_faces,
                                self.uc, self.amp, self.seed, self.half, self.profile)

    def fields_torch(self, device):
        return initial_velocity_torch(self.nx, self.ny, self.nz, self.y_faces, self.uc,
                                      self.amp, self.seed, self.half, device, self.profile)


def _sphere_body(level, radius, c0, U):
    V, F = icosphere(level)
    c0 = np.asarray(c0, np.float64)
    U = np.asarray(U, np.float64)
    return Body("rigid", V * radius, F, lambda t: sphere_translation(t, c0, U))


def config(name: str) -> Workload:
    """Named synthetic workloads.

    c1   64x48x64 uniform channel, Re 100, dt 1e-3, 10 steps; one sphere of
         diameter 0.5 (1280 triangles) translating at (0.5, 0, 0).
    c2   256x192x256 tanh-stretched channel, Re 1000, dt 1e-3, 100 steps; a
         zero-thickness 1.0 x 0.6 plate (1920 triangles) heaving
         0.2 sin(2 pi t) and pitching +-15 deg at twice the frequency.
    c3   512x384x512 stretched channel, Re 2000, dt 1e-3, 200 steps; a
         deforming closed body r = 0.4 (1 + 0.1 Y20 sin 4 pi t), 20480 tris.
    c5   1024x768x1024 stretched channel, Re 2800, dt 1e-3, 50 steps; 64
         translating spheres (1280 tris each) and 3 hinged rotating
         leaflets (10000 tris each), 111920 triangles.
    tiny  small ragged grids for parity tests (several tiles plus a tail).
    """
    two_pi, pi = 2.0 * math.pi, math.pi
    if name == "c1":
        ny = 48
        return Workload("c1", 64, ny, 64, two_pi, pi, uniform_faces(ny), 100.0,
                        1e-3, 10, 1.0, 0.01, 1, -2.0 / 100.0,
                        [_sphere_body(3, 0.25, (pi, 0.0, 0.5 * pi), (0.5, 0.0, 0.0))])
    if name == "c2":
        ny = 192
        V, F = plate_mesh(1.0, 0.6, 40, 24)
        return Workload("c2", 256, ny, 256, two_pi, pi, tanh_faces(ny, 2.0), 1000.0,
                        1e-3, 100, 1.0, 0.01, 2, -2.0 / 1000.0,
                        [Body("rigid", V, F, plate_heave_pitch)])
    if name == "c3":
        ny = 384
        V, F = icosphere(5)
        c = (pi, 0.0, 0.5 * pi)
        return Workload("c3", 512, ny, 512, two_pi, pi, tanh_faces(ny, 2.0), 2000.0,
                        1e-3, 200, 1.0, 0.01, 3, -2.0 / 2000.0,
                        [Body("deform", deform_vertex_data(V, 0.4), F,
                              lambda t: deform_coef(t, c, 0.4))])
    if name == "c5":
        # 1024x768x1024 stretched channel, Re 2800 (bulk Reynolds number 5600
        # on the channel height), centre velocity 1.5 (bulk 1) plus a 0.1
        # perturbation, 50 steps of 1e-3; a constant driving gradient of the
        # laminar profile stands in for constant-flow-rate control
        ny = 768
        return Workload("c5", 1024, ny, 1024, two_pi, pi, tanh_faces(ny, 2.0), 2800.0,
                        1e-3, 50, 1.5, 0.1, 5, -2.0 * 1.5 / 2800.0, c5_bodies())
    if name == "plane":
        return plane_channel(180)
    if name == "turb":
        return turbulent_plane_channel()
    if name == "tiny":
        # ragged, non-power-of-two sizes: 40 = 8*5 and 36 = 4*9 exercise the
        # mixed-radix transforms; the sphere spans several tiles.
        ny = 30
        return Workload("tiny", 40, ny, 36, two_pi, pi, tanh_faces(ny, 1.5), 100.0,
                        2e-3, 3, 1.0, 0.05, 7, -2.0 / 100.0,
                        [_sphere_body(2, 0.5, (3.0, 0.0, 1.6), (0.3, 0.1, -0.2))])
    if name == "tiny_plate":
        ny = 32
        V, F = plate_mesh(1.2, 0.8, 10, 6)
        return Workload("tiny_plate", 48, ny, 40, two_pi, pi, tanh_faces(ny, 2.0), 200.0,
                        2e-3, 3, 1.0, 0.02, 11, -2.0 / 200.0,
                        [Body("rigid", V, F, plate_heave_pitch)])
    raise KeyError(name)


def _full_span_plane(lx, lz, y0, nq_x, nq_z):
    P, T = plate_mesh(lx, lz, nq_x, nq_z)
    centre = (0.5 * lx, y0, 0.5 * lz)
    return Body("rigid", P, T, lambda t: sphere_translation(t, centre, (0.0, 0.0, 0.0)))


def plane_channel(N: int = 180) -> Workload:
    """Sec. 4.2: the channel x in [-1, 1) (here [0, 2)), z likewise, y in
    [-1/4, 2] with no-slip walls, split by a full-span immersed plane near
    y = 0; above it a driving force (plane Poiseuille flow of centre velocity
    1 between the plane and y = 2, Re 100), below it the wall-normal vortex
    forcing F_y = 50 sin(pi (y + 1/4)/(1/4)) cos(pi x).  Uniform spacing
    Delta = 2/N; the plane sits at y0 = 0.37 Delta, off every node (the
    paper scales the lower grid for the same purpose).  Starts from the
    exact upper profile, zero below."""
    d = 2.0 / N
    ny = int(round(2.25 / d))
    yf = uniform_faces(ny, -0.25, 2.0)
    y0 = 0.37 * d
    prof = lambda y: np.where(y > y0, (y - y0) * (2.0 - y) / ((1.0 - 0.5 * y0) ** 2), 0.0)
    wl = Workload("plane", N, ny, N, 2.0, 2.0, yf, 100.0, 0.25 * d, 100, 1.0, 0.0, 6, 0.0,
                  [_full_span_plane(2.0, 2.0, y0, N // 4, N // 4)], profile=prof, vforce="vortex")
    return wl


def _cluster_faces(n: int, y0: float, y1: float, beta: float = 1.6) -> np.ndarray:
    """n+1 faces on [y0, y1] clustered at both ends (tanh)."""
    j = np.arange(n + 1, dtype=np.float64)
    s = np.tanh(beta * (2.0 * j / n - 1.0)) / math.tanh(beta)
    yf = y0 + 0.5 * (y1 - y0) * (s + 1.0)
    yf[0], yf[-1] = y0, y1
    return yf


def turbulent_plane_channel() -> Workload:
    """Sec. 4.3: x in [0, 4 pi), z in [0, 2 pi) (256 x 256 points), y in
    [-1/4, 2]: 127 cells clustered at the plane and at y = 2 above it, 31
    uniform cells below; Re_tau = 200 (u_tau = delta = 1), AB2 + CN; a
    driving force 1 (= u_tau^2/delta) above the plane and the relaxation
    F_y = -5 (v - 1) below it.  The plane lies at 0.37 of the first upper
    cell, off every node (the paper's formula for the upper grid is
    garbled; tanh clustering stands in for it).  Starts from a turbulent-like
    mean profile (centre velocity 18) with a 1.0 perturbation."""
    upper = _cluster_faces(127, 0.0, 2.0)
    lower = uniform_faces(31, -0.25, 0.0)
    yf = np.concatenate([lower[:-1], upper])
    y0 = 0.37 * (upper[1] - upper[0])
    prof = lambda y: np.where(y > y0, 18.0 * (1.0 - (y - 1.0) ** 2), 0.0)
    lx, lz = 4.0 * math.pi, 2.0 * math.pi
    return Workload("turb", 256, 158, 256, lx, lz, yf, 200.0, 5e-4, 100, 1.0, 1.0, 7, 0.0,
                    [_full_span_plane(lx, lz, y0, 64, 32)], scheme="ab2", profile=prof,
                    vforce="relax")


def volume_force(wl: Workload, comp: int):
    """(f0, kappa) of component comp of the immersed-plane channels on its
    lattice ([y][z][x] numpy arrays; kappa None where it vanishes), or
    (None, None) for a workload without volume force."""
    if wl.vforce is None:
        return None, None
    dx, dz = wl.lx / wl.nx, wl.lz / wl.nz
    yf = np.asarray(wl.y_faces, np.float64)
    ox, oz = {0: (0.0, 0.5), 1: (0.5, 0.5), 2: (0.5, 0.0)}[comp]
    ys = yf if comp == 1 else 0.5 * (yf[:-1] + yf[1:])
    x = (np.arange(wl.nx) + ox) * dx
    z = (np.arange(wl.nz) + oz) * dz
    Y, _, X = np.meshgrid(ys, z, x, indexing="ij")
    lo = float(yf[0])
    body_y = float(wl.bodies[0].coef(0.0)[1])     # the plane's height
    f0 = np.zeros(Y.shape)
    kappa = None
    if comp == 0:
        drive = 2.0 / (wl.re * (1.0 - 0.5 * body_y) ** 2) if wl.vforce == "vortex" else 1.0
        f0[Y > body_y] = drive
    elif comp == 1:
        below = (Y > lo) & (Y < 0.0)
        if wl.vforce == "vortex":
            f0[below] = (50.0 * np.sin(np.pi * (Y - lo) / (-lo)) * np.cos(np.pi * X))[below]
        else:
            f0[below] = 5.0
            kappa = np.where(below, -5.0, 0.0)
    return f0, kappa


def leaflet_mesh(radius: float, chord: float, span: float, n_arc: int, n_span: int):
    """Zero-thickness leaflet: a cylindrical arc in the x-y plane (radius
    `radius`, chord `chord`) extruded along z over `span`, with one edge on
    the z axis (its hinge).  The arc rises from the hinge along +y, bulging
    towards -x.  n_arc x n_span quads, 2 triangles each.  Returns (verts
    relative to the hinge centre, tris)."""
    ang = 2.0 * math.asin(0.5 * chord / radius)
    ph = ang * np.arange(n_arc + 1, dtype=np.float64) / n_arc
    zs = -0.5 * span + span * np.arange(n_span + 1, dtype=np.float64) / n_span
    x = -radius + radius * np.cos(ph)
    y = radius * np.sin(ph)
    X = np.repeat(x, n_span + 1)
    Y = np.repeat(y, n_span + 1)
    Z = np.tile(zs, n_arc + 1)
    V = np.stack([X, Y, Z], axis=1)
    tris = []
    for a in range(n_arc):
        for b in range(n_span):
            v00 = a * (n_span + 1) + b
            v10 = (a + 1) * (n_span + 1) + b
            tris.append((v00, v10, v10 + 1))
            tris.append((v00, v10 + 1, v00 + 1))
    return V, np.array(tris, dtype=np.int32)


def leaflet_rotation(t: float, hinge) -> np.ndarray:
    """Rigid rotation of a leaflet about the z axis through its hinge:
    theta(t) = (pi/3) (1 - cos(2 pi (t + 1/4)))/2."""
    w = 2.0 * math.pi
    th = (math.pi / 3.0) * 0.5 * (1.0 - math.cos(w * (t + 0.25)))
    thd = (math.pi / 3.0) * 0.5 * w * math.sin(w * (t + 0.25))
    ct, st = math.cos(th), math.sin(th)
    R = [[ct, -st, 0.0], [st, ct, 0.0], [0.0, 0.0, 1.0]]
    return rigid_coef(hinge, R, (0.0, 0.0, 0.0), (0.0, 0.0, thd))


def c5_bodies(seed: int = 5, nspheres: int = 64, h: float = 0.016):
    """Bodies of the large multi-body workload: three leaflets (10000
    triangles each) hinged along z at (x_h, -0.3) for x_h = pi/2, pi, 3 pi/2
    and spanning z in [0.57, 2.57], and `nspheres` spheres of diameter 0.1
    (1280 triangles) with centres at |y| <= 0.8, at least 2h apart from each
    other and clear of the leaflets' swept region, each translating at a
    speed drawn from U[0, 1] in a random direction."""
    rng = np.random.default_rng(seed)
    bodies = []
    hinges = [(0.5 * math.pi, -0.3, 1.57), (math.pi, -0.3, 1.57), (1.5 * math.pi, -0.3, 1.57)]
    V, F = leaflet_mesh(0.3, 0.3, 2.0, 50, 100)
    for hg in hinges:
        bodies.append(Body("rigid", V, F, lambda t, hg=hg: leaflet_rotation(t, hg)))
    r = 0.05
    centres = []
    while len(centres) < nspheres:
        c = np.array([rng.uniform(0.0, 2.0 * math.pi), rng.uniform(-0.8, 0.8),
                      rng.uniform(0.0, math.pi)])
        # clear of the leaflets (|x - x_h| < 0.45 within their y and z range)
        near_leaflet = any(abs(c[0] - hg[0]) < 0.45 and -0.75 < c[1] < 0.15 and
                           0.4 < c[2] < 2.75 for hg in hinges)
        if near_leaflet:
            continue
        if all(np.linalg.norm(c - o) >= 2 * r + 2 * h for o in centres):
            centres.append(c)
    for c in centres:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        bodies.append(_sphere_body(3, r, c, float(rng.uniform(0.0, 1.0)) * d))
    return bodies


CONFIG_NAMES = ("c1", "c2", "c3", "c5", "tiny", "tiny_plate")


def _plate_fixed(chord, span, nq_x, nq_z, c0, U, theta):
    """Zero-thickness plate pitched by a fixed angle theta about z,
    translating at constant velocity U from c0."""
    V, F = plate_mesh(chord, span, nq_x, nq_z)
    ct, st = math.cos(theta), math.sin(theta)
    R = np.array([[ct, -st, 0.0], [st, ct, 0.0], [0.0, 0.0, 1.0]])
    c0 = np.asarray(c0, np.float64)
    U = np.asarray(U, np.float64)
    return Body("rigid", V, F, lambda t: rigid_coef(c0 + U * t, R, U, np.zeros(3)))


# quads (m, n) of the batch plates for 2*m*n triangles
_PLATE_QUADS = {320: (16, 10), 640: (20, 16), 1280: (32, 20), 2560: (40, 32), 5120: (64, 40)}


def batch_sim(s: int, steps: int = 20) -> Workload:
    """Simulation s of the batched workload (seed 4000 + s).

    Fixed-spacing box: uniform spacing 1/32 in every direction, nx, nz drawn
    from {32, 48, ..., 128} and ny from {32, 48, ..., 96} (multiples of 16, so
    the transform radices are 2, 3, 5, 7); Lx = nx/32, Lz = nz/32, walls at
    y = -Ly/2 and +Ly/2 with Ly = ny/32.  Re 100, dt 1e-3, Poiseuille flow of
    centre velocity 1 plus a 0.01 perturbation.  One body, its type drawn
    uniformly: a sphere (level 2..4, diameter 0.3..0.5), a plate (chord and
    span 0.3..0.6, 320..5120 triangles, pitched by a fixed angle within +-15
    deg) or a deforming closed body (the law of the large deforming case,
    r0 0.15..0.25, level 2..4), each translating at a speed drawn from
    U[0, 1] in a random direction.  The centre is uniform in the box with a
    wall clearance of at least r + h + 2 d0 + steps dt |U| (h = 2 sqrt(3) d0
    the probe length), so that the body stays clear of the walls over
    `steps` steps; where the channel is too narrow for that, the speed is
    lowered until it fits."""
    rng = np.random.default_rng(4000 + s)
    d0 = 1.0 / 32.0
    nx = int(rng.choice(np.arange(32, 129, 16)))
    nz = int(rng.choice(np.arange(32, 129, 16)))
    ny = int(rng.choice(np.arange(32, 97, 16)))
    lx, lz, ly = nx * d0, nz * d0, ny * d0
    half = 0.5 * ly
    yf = uniform_faces(ny, -half, half)
    re, dt = 100.0, 1e-3
    h = 2.0 * math.sqrt(3.0) * d0
    kind = int(rng.integers(3))
    speed = float(rng.uniform(0.0, 1.0))
    dirn = rng.standard_normal(3)
    dirn /= np.linalg.norm(dirn)
    U = speed * dirn
    if kind == 0:
        level = int(rng.integers(2, 5))
        r = 0.5 * float(rng.uniform(0.3, 0.5))
    elif kind == 1:
        chord = float(rng.uniform(0.3, 0.6))
        span = float(rng.uniform(0.3, 0.6))
        ntri = int(rng.choice(sorted(_PLATE_QUADS)))
        theta = float(rng.uniform(-1.0, 1.0)) * math.pi / 12.0
        r = 0.5 * max(chord, span)
    else:
        level = int(rng.integers(2, 5))
        r0 = float(rng.uniform(0.15, 0.25))
        r = r0 * 1.07
    room = 0.95 * half - (r + h + 2.0 * d0)
    if steps * dt * float(np.linalg.norm(U)) > room:
        U = U * (max(room, 0.0) / (steps * dt * float(np.linalg.norm(U))))
    clear = r + h + 2.0 * d0 + steps * dt * float(np.linalg.norm(U))
    c = np.array([rng.uniform(0.0, lx), rng.uniform(-half + clear, half - clear),
                  rng.uniform(0.0, lz)])
    if kind == 0:
        body = _sphere_body(level, r, c, U)
    elif kind == 1:
        m, n = _PLATE_QUADS[ntri]
        body = _plate_fixed(chord, span, m, n, c, U, theta)
    else:
        V, F = icosphere(level)
        cc = tuple(c)
        Ut = tuple(float(x) for x in U)
        body = Body("deform", deform_vertex_data(V, r0), F,
                    lambda t, cc=cc, r0=r0, Ut=Ut: deform_coef(t, cc, r0, U=Ut))
    dpdx = -2.0 * 1.0 / (re * half * half)
    return Workload(f"c4.{s}", nx, ny, nz, lx, lz, yf, re, dt, steps, 1.0, 0.01, 4000 + s,
                    dpdx, [body], half=half)


def batch(nsim: int = 64, steps: int = 20):
    """The batched workload: simulations 0..nsim-1 of batch_sim."""
    return [batch_sim(s, steps) for s in range(nsim)]
