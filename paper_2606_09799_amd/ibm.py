"""Thin ctypes binding of libibm (include/ibm.h): argument marshalling only.

Every computation happens in the HIP kernels of libibm.so; this module checks
shapes, dtypes and devices of torch tensors (PyTorch supplies only device
memory and the stream) and forwards raw pointers.  If the library has not
been built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2606_09799_amd.build` (no CPU fallback exists)")
_lib = ctypes.CDLL(LIB_PATH)

IBM_OK, IBM_EINVAL, IBM_ENOMEM, IBM_EHIP, IBM_ECAPACITY = 0, -1, -2, -3, -4
IBM_ENONFINITE, IBM_ECFL, IBM_EGEOM, IBM_ECOMPAT = -5, -6, -7, -8
FLAG_CAPACITY, FLAG_NONFINITE, FLAG_GEOM, FLAG_REFINE = 1, 2, 4, 8
FLAG_CFL, FLAG_COMPAT = 16, 32
IBM_REFINE_STATS = 6
IBM_RIGID_STATE, IBM_RIGID_PROPS = 28, 8
IBM_FP64, IBM_MIXED = 0, 1
IBM_RK2CN, IBM_AB2CN = 0, 1
IBM_Q_NONE, IBM_Q_UNIFORM, IBM_Q_ENERGY = 0, 1, 2


class IbmGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("reserved", c_int32),
                ("lx", c_double), ("lz", c_double), ("y_faces", POINTER(c_double))]


class IbmOpts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("scheme", c_int32), ("re", c_double),
                ("dpdx", c_double), ("force_cap", c_int64), ("use_q", c_int32),
                ("refine_max", c_int32), ("refine_tol", c_double),
                ("mixed_poisson", c_int32), ("reserved", c_int32)]


class IbmBody(ctypes.Structure):
    _fields_ = [("nv", c_int32), ("nt", c_int32), ("xyz", c_void_p), ("vel", c_void_p),
                ("tri", c_void_p)]


class IbmTags(ctypes.Structure):
    _fields_ = [("idx", c_void_p * 3), ("tri", c_void_p * 3), ("cb", c_void_p),
                ("count", c_void_p), ("mask", c_void_p * 3), ("cb_mask", c_void_p),
                ("capacity", c_int64)]


class IbmState(ctypes.Structure):
    _fields_ = [("u", c_void_p), ("v", c_void_p), ("w", c_void_p), ("p", c_void_p),
                ("h", c_void_p * 3)]


class IbmSim(ctypes.Structure):
    _fields_ = [("state", IbmState), ("motion", c_int32), ("nv", c_int32), ("nt", c_int32),
                ("ref", c_void_p), ("xyz", c_void_p), ("vel", c_void_p), ("tri", c_void_p)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_create = _sig("ibm_create", c_int32, POINTER(IbmGrid), POINTER(IbmOpts), c_void_p,
               POINTER(c_void_p))
_destroy = _sig("ibm_destroy", None, c_void_p)
_set_stream = _sig("ibm_set_stream", c_int32, c_void_p, c_void_p)
_body_rigid = _sig("ibm_body_rigid", c_int32, c_void_p, c_void_p, c_int32, POINTER(c_double),
                   c_void_p, c_void_p)
_body_deform = _sig("ibm_body_deform", c_int32, c_void_p, c_void_p, c_int32, POINTER(c_double),
                    c_void_p, c_void_p)
_tag = _sig("ibm_tag", c_int32, c_void_p, POINTER(IbmBody), c_int32, POINTER(IbmTags))
_count_host = _sig("ibm_tags_count_host", c_int32, c_void_p, POINTER(c_int64))
_tags_copy = _sig("ibm_tags_copy", c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_int64)
_force = _sig("ibm_force", c_int32, c_void_p, c_void_p, c_void_p, c_void_p)
_viscous = _sig("ibm_viscous", c_int32, c_void_p, c_void_p, POINTER(c_void_p),
                POINTER(c_void_p), c_double, c_double, c_double, c_void_p, c_void_p, c_void_p)
_mass_rhs = _sig("ibm_mass_rhs", c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                 c_double, c_void_p, c_void_p)
_poisson = _sig("poisson_solve", c_int32, c_void_p, c_void_p, c_void_p)
_project = _sig("ibm_project", c_int32, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                c_void_p, c_void_p)
_step = _sig("ibm_step", c_int32, c_void_p, POINTER(IbmState), POINTER(IbmBody), c_int32,
             c_double)
_refine_stats = _sig("ibm_refine_stats", c_int32, c_void_p, POINTER(c_double), c_int32)
_batch_create = _sig("ibm_batch_create", c_int32, POINTER(IbmGrid), POINTER(IbmOpts),
                     POINTER(IbmSim), c_int32, c_void_p, POINTER(c_void_p))
_batch_destroy = _sig("ibm_batch_destroy", None, c_void_p)
_batch_context = _sig("ibm_batch_context", c_void_p, c_void_p, c_int32)
_batch_step = _sig("ibm_batch_step", c_int32, c_void_p, POINTER(c_double), c_double, c_int32)
_batch_check = _sig("ibm_batch_check", c_int32, c_void_p, POINTER(c_uint32))


class IbmBatchPlan(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("streams", c_int32), ("rhs_planes", c_int32),
                ("reserved", c_int32), ("ms_per_step", c_double)]


_batch_set_plan = _sig("ibm_batch_set_plan", c_int32, c_void_p, POINTER(IbmBatchPlan))
_batch_get_plan = _sig("ibm_batch_get_plan", c_int32, c_void_p, POINTER(IbmBatchPlan))
_batch_tune = _sig("ibm_batch_tune", c_int32, c_void_p, POINTER(c_double), c_double, c_int32,
                   c_void_p, c_int64, POINTER(IbmBatchPlan), POINTER(IbmBatchPlan), c_int32,
                   POINTER(c_int32))
_batch_tune_bytes = _sig("ibm_batch_tune_scratch_bytes", c_int64, c_void_p)
_poisson_static = _sig("poisson_solve_static", c_int32, POINTER(IbmGrid), c_void_p, c_void_p,
                       c_void_p)
_check = _sig("ibm_check", c_int32, c_void_p, POINTER(c_uint32))
_noslip = _sig("ibm_noslip_error", c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
               POINTER(c_double))
_pressure_cb = _sig("ibm_pressure_cb", c_int32, c_void_p, c_void_p, c_void_p, c_int64)
_vforce = _sig("ibm_set_volume_force", c_int32, c_void_p, c_int32, c_void_p, c_void_p)
_body_rigid_dev = _sig("ibm_body_rigid_dev", c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                       c_void_p, c_void_p)
_rigid_advance = _sig("ibm_rigid_advance", c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                      c_void_p, c_double, c_void_p)
_loads = _sig("ibm_loads", c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
              c_void_p, c_void_p, c_void_p)
_divergence = _sig("ibm_divergence", c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                   POINTER(c_double))
_strerror = _sig("ibm_strerror", c_char_p, c_int32)
_profile = _sig("ibm_profile", c_int32, c_void_p, c_int32, c_char_p)
_profile_read = _sig("ibm_profile_read", c_int32, c_void_p, c_char_p, c_int32,
                     POINTER(c_int64), POINTER(c_double), c_int32)

EXPORTS = ("ibm_create", "ibm_destroy", "ibm_set_stream", "ibm_body_rigid", "ibm_body_deform",
           "ibm_tag", "ibm_tags_count_host", "ibm_tags_copy", "ibm_force", "ibm_viscous",
           "ibm_mass_rhs", "poisson_solve", "ibm_project", "ibm_step", "ibm_refine_stats",
           "ibm_check", "ibm_strerror", "ibm_profile", "ibm_profile_read",
           "ibm_batch_create", "ibm_batch_destroy", "ibm_batch_context", "ibm_batch_step",
           "ibm_batch_check", "ibm_batch_set_plan", "ibm_batch_get_plan", "ibm_batch_tune",
           "ibm_batch_tune_scratch_bytes", "poisson_solve_static",
           "ibm_noslip_error", "ibm_pressure_cb", "ibm_divergence", "ibm_loads",
           "ibm_set_volume_force", "ibm_body_rigid_dev", "ibm_rigid_advance")
COEF_STRIDE = 18
BATCH_SERIAL, BATCH_STREAMS, BATCH_GRAPH, BATCH_PLAN, BATCH_GROUPED = 0, 1, 2, 3, 4
_MODE_NAMES = {BATCH_STREAMS: "streams", BATCH_GRAPH: "graph", BATCH_GROUPED: "grouped"}
MOTION_RIGID, MOTION_DEFORM = 0, 1


class IbmError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {code} ({_strerror(code).decode()})")
        self.code = code


def _ok(code, where):
    if code != IBM_OK:
        raise IbmError(code, where)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, numel, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


class Context:
    """One grid on the current device, bound to torch's current stream.
    precision: "fp64", or "mixed" (p and H in float32; u, v, w in float64);
    mixed_poisson: "fp64" or "refined" (FP32 transforms refined with FP64
    residuals) for the mixed form.
    use_q: True (uniform q_F), "energy" (mass- and energy-conserving shape)
    or False (standard projection)."""

    def __init__(self, nx, ny, nz, lx, lz, y_faces, re, dpdx=0.0, scheme="rk2", use_q=True,
                 force_cap=0, precision="fp64", refine_max=0, refine_tol=0.0,
                 mixed_poisson="fp64"):
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision: 'fp64' or 'mixed'")
        self.precision = precision
        # dtype of p and of the H arrays
        self.pdtype = torch.float32 if precision == "mixed" else torch.float64
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.cells = self.nx * self.ny * self.nz
        self.vfaces = self.nx * (self.ny + 1) * self.nz
        yf = np.ascontiguousarray(np.asarray(y_faces, dtype=np.float64))
        if yf.shape != (self.ny + 1,):
            raise ValueError("y_faces must hold ny+1 values")
        self._yf = yf
        g = IbmGrid(self.nx, self.ny, self.nz, 0, float(lx), float(lz),
                    yf.ctypes.data_as(POINTER(c_double)))
        qmode = IBM_Q_ENERGY if use_q == "energy" else (IBM_Q_UNIFORM if use_q else IBM_Q_NONE)
        o = IbmOpts(IBM_MIXED if precision == "mixed" else IBM_FP64,
                    IBM_RK2CN if scheme == "rk2" else IBM_AB2CN, float(re),
                    float(dpdx), int(force_cap), qmode, int(refine_max),
                    float(refine_tol), 1 if mixed_poisson == "refined" else 0, 0)
        h = c_void_p()
        _ok(_create(ctypes.byref(g), ctypes.byref(o), _stream(), ctypes.byref(h)), "ibm_create")
        self.handle = h
        self.re = float(re)

    def close(self):
        if self.handle:
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def comp_numel(self, c):
        return self.vfaces if c == 1 else self.cells

    def bind_current_stream(self):
        _ok(_set_stream(self.handle, _stream()), "ibm_set_stream")


class Body:
    """Device arrays of one triangulated surface (f64 vertices/velocities,
    i32 triangles)."""

    def __init__(self, xyz, vel, tri):
        self.xyz, self.vel, self.tri = xyz, vel, tri
        self.nv = xyz.shape[0]
        self.nt = tri.shape[0]

    def desc(self):
        return IbmBody(self.nv, self.nt, _dev(self.xyz, torch.float64, 3 * self.nv, "xyz"),
                       _dev(self.vel, torch.float64, 3 * self.nv, "vel"),
                       _dev(self.tri, torch.int32, 3 * self.nt, "tri"))


def _bodies(bodies):
    arr = (IbmBody * max(1, len(bodies)))()
    for i, b in enumerate(bodies):
        arr[i] = b.desc()
    return arr, len(bodies)


def ibm_body_rigid(ctx, x0, coef, xyz, vel):
    nv = x0.shape[0]
    cf = np.ascontiguousarray(np.asarray(coef, np.float64))
    if cf.shape != (18,):
        raise ValueError("rigid coefficients: 18 values")
    _ok(_body_rigid(ctx.handle, _dev(x0, torch.float64, 3 * nv, "x0"), nv,
                    cf.ctypes.data_as(POINTER(c_double)), _dev(xyz, torch.float64, 3 * nv, "xyz"),
                    _dev(vel, torch.float64, 3 * nv, "vel")), "ibm_body_rigid")


def ibm_body_deform(ctx, data, coef, xyz, vel):
    nv = data.shape[0]
    cf = np.ascontiguousarray(np.asarray(coef, np.float64))
    if cf.shape != (9,):
        raise ValueError("deform coefficients: 9 values")
    _ok(_body_deform(ctx.handle, _dev(data, torch.float64, 4 * nv, "data"), nv,
                     cf.ctypes.data_as(POINTER(c_double)),
                     _dev(xyz, torch.float64, 3 * nv, "xyz"),
                     _dev(vel, torch.float64, 3 * nv, "vel")), "ibm_body_deform")


def ibm_tag(ctx, bodies):
    arr, n = _bodies(bodies)
    t = IbmTags()
    _ok(_tag(ctx.handle, arr, n, ctypes.byref(t)), "ibm_tag")
    return t


def ibm_tags_count_host(ctx):
    out = (c_int64 * 4)()
    _ok(_count_host(ctx.handle, out), "ibm_tags_count_host")
    return [int(x) for x in out]


def tag_lists(ctx):
    """Copies of the last tagging: ([(idx i64, tri i32)] per component, cb i64)
    as CUDA tensors (synchronises once for the counts)."""
    counts = ibm_tags_count_host(ctx)
    out = []
    for c in range(3):
        n = counts[c]
        idx = torch.empty(n, dtype=torch.int64, device="cuda")
        tri = torch.empty(n, dtype=torch.int32, device="cuda")
        _ok(_tags_copy(ctx.handle, c, c_void_p(idx.data_ptr()) if n else None,
                       c_void_p(tri.data_ptr()) if n else None, n), "ibm_tags_copy")
        out.append((idx, tri))
    n = counts[3]
    cb = torch.empty(n, dtype=torch.int64, device="cuda")
    _ok(_tags_copy(ctx.handle, 3, c_void_p(cb.data_ptr()) if n else None, None, n),
        "ibm_tags_copy")
    return out, cb


def ibm_force(ctx, u, v, w):
    _ok(_force(ctx.handle, _dev(u, torch.float64, ctx.cells, "u"),
               _dev(v, torch.float64, ctx.vfaces, "v"),
               _dev(w, torch.float64, ctx.cells, "w")), "ibm_force")


def _ptr3(ts, ctx, name):
    if ts is None:
        return None
    arr = (c_void_p * 3)()
    for c in range(3):
        arr[c] = _dev(ts[c], ctx.pdtype, ctx.comp_numel(c), f"{name}[{c}]")
    return arr


def ibm_viscous(ctx, p, h_prev, h_out, gamma, rho, dt, u, v, w):
    _ok(_viscous(ctx.handle, _dev(p, ctx.pdtype, ctx.cells, "p"), _ptr3(h_prev, ctx, "h_prev"),
                 _ptr3(h_out, ctx, "h_out"), float(gamma), float(rho), float(dt),
                 _dev(u, torch.float64, ctx.cells, "u"), _dev(v, torch.float64, ctx.vfaces, "v"),
                 _dev(w, torch.float64, ctx.cells, "w")), "ibm_viscous")


def ibm_noslip_error(ctx, u, v, w):
    """No-slip error at the forcing nodes of the last tagging: (mean of the
    three components, [u, v, w] means of |error|)."""
    eps = (c_double * 4)()
    _ok(_noslip(ctx.handle, _dev(u, torch.float64, ctx.cells, "u"),
                _dev(v, torch.float64, ctx.vfaces, "v"), _dev(w, torch.float64, ctx.cells, "w"),
                eps), "ibm_noslip_error")
    return eps[0], [eps[1], eps[2], eps[3]]


def ibm_body_rigid_dev(ctx, x0, coef, xyz, vel):
    """ibm_body_rigid with the coefficients in a float64 device tensor (18)."""
    nv = x0.shape[0]
    _ok(_body_rigid_dev(ctx.handle, _dev(x0, torch.float64, 3 * nv, "x0"), nv,
                        _dev(coef, torch.float64, 18, "coef"),
                        _dev(xyz, torch.float64, 3 * nv, "xyz"),
                        _dev(vel, torch.float64, 3 * nv, "vel")), "ibm_body_rigid_dev")


def ibm_rigid_advance(ctx, state, props, loads, dt, coef):
    """One AB2 step of nb free rigid bodies: state (nb, IBM_RIGID_STATE),
    props (nb, IBM_RIGID_PROPS), loads (nb, 6), coef (nb, 18) float64 device
    tensors."""
    nb = loads.numel() // 6
    _ok(_rigid_advance(ctx.handle, nb, _dev(state, torch.float64, nb * IBM_RIGID_STATE, "state"),
                       _dev(props, torch.float64, nb * IBM_RIGID_PROPS, "props"),
                       _dev(loads, torch.float64, 6 * nb, "loads"), float(dt),
                       _dev(coef, torch.float64, 18 * nb, "coef")), "ibm_rigid_advance")


def ibm_set_volume_force(ctx, comp, f0=None, kappa=None):
    """Volume force f0 + kappa u_comp on component comp (float64 device
    tensors on its lattice, or None); the context keeps references to them."""
    numel = ctx.comp_numel(comp)
    _ok(_vforce(ctx.handle, int(comp), _dev(f0, torch.float64, numel, "f0"),
                _dev(kappa, torch.float64, numel, "kappa")), "ibm_set_volume_force")
    if not hasattr(ctx, "_vforce"):
        ctx._vforce = {}
    ctx._vforce[comp] = (f0, kappa)


def ibm_loads(ctx, u, v, w, p, sides, pole, traction, loads):
    """Hydrodynamic loads (Sec. 3.3) of the bodies of the last tagging.
    sides: i32 device tensor (nb,), 2 for a two-sided body; pole: f64 (nb, 3);
    traction: f64 (ntri, 3) per marker; loads: f64 (nb, 6), force and torque."""
    nb = sides.numel()
    _ok(_loads(ctx.handle, _dev(u, torch.float64, ctx.cells, "u"),
               _dev(v, torch.float64, ctx.vfaces, "v"), _dev(w, torch.float64, ctx.cells, "w"),
               _dev(p, ctx.pdtype, ctx.cells, "p"), _dev(sides, torch.int32, nb, "sides"),
               _dev(pole, torch.float64, 3 * nb, "pole"),
               _dev(traction, torch.float64, traction.numel(), "traction"),
               _dev(loads, torch.float64, 6 * nb, "loads")), "ibm_loads")


def ibm_pressure_cb(ctx, p, out):
    """Pressure reconstructed on the boundary cells of the last tagging into
    out (f64 device tensor, one value per boundary cell, ascending)."""
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out: contiguous float64 device tensor")
    _ok(_pressure_cb(ctx.handle, _dev(p, ctx.pdtype, ctx.cells, "p"), c_void_p(out.data_ptr()),
                     out.numel()), "ibm_pressure_cb")


def ibm_mass_rhs(ctx, u, v, w, alpha_dt, rhs, qf=None, p=None):
    """qf: 1 value (q_F), or 2 (c0, c1) for the energy-conserving shape,
    which also needs p."""
    _ok(_mass_rhs(ctx.handle, _dev(u, torch.float64, ctx.cells, "u"),
                  _dev(v, torch.float64, ctx.vfaces, "v"),
                  _dev(w, torch.float64, ctx.cells, "w"), _dev(p, ctx.pdtype, ctx.cells, "p"),
                  float(alpha_dt), _dev(rhs, torch.float64, ctx.cells, "rhs"),
                  _dev(qf, torch.float64, None, "qf")), "ibm_mass_rhs")


def ibm_divergence(ctx, u, v, w):
    """Post-projection divergence: (max over C_F of |D u - q_F|, q_F)."""
    out = (c_double * 2)()
    _ok(_divergence(ctx.handle, _dev(u, torch.float64, ctx.cells, "u"),
                    _dev(v, torch.float64, ctx.vfaces, "v"),
                    _dev(w, torch.float64, ctx.cells, "w"), out), "ibm_divergence")
    return out[0], out[1]


def poisson_solve_static(nx, ny, nz, lx, lz, y_faces, rhs, phi):
    """poisson_solve_static: the FP64 Poisson solve with no context, its
    workspace in the library's static device array (nothing is allocated);
    enqueued on torch's current stream.  rhs, phi: float64 device tensors of
    nx*ny*nz values."""
    yf = np.ascontiguousarray(np.asarray(y_faces, dtype=np.float64))
    if yf.shape != (int(ny) + 1,):
        raise ValueError("y_faces must hold ny+1 values")
    g = IbmGrid(int(nx), int(ny), int(nz), 0, float(lx), float(lz),
                yf.ctypes.data_as(POINTER(c_double)))
    cells = int(nx) * int(ny) * int(nz)
    _ok(_poisson_static(ctypes.byref(g), _dev(rhs, torch.float64, cells, "rhs"),
                        _dev(phi, torch.float64, cells, "phi"), _stream()), "poisson_solve_static")


def poisson_solve(ctx, rhs, phi):
    _ok(_poisson(ctx.handle, _dev(rhs, torch.float64, ctx.cells, "rhs"),
                 _dev(phi, torch.float64, ctx.cells, "phi")), "poisson_solve")


def ibm_project(ctx, phi, alpha_dt, u, v, w, p):
    _ok(_project(ctx.handle, _dev(phi, torch.float64, ctx.cells, "phi"), float(alpha_dt),
                 _dev(u, torch.float64, ctx.cells, "u"), _dev(v, torch.float64, ctx.vfaces, "v"),
                 _dev(w, torch.float64, ctx.cells, "w"),
                 _dev(p, ctx.pdtype, ctx.cells, "p")), "ibm_project")


def ibm_step(ctx, u, v, w, p, bodies, dt, h=None):
    st = IbmState(_dev(u, torch.float64, ctx.cells, "u"), _dev(v, torch.float64, ctx.vfaces, "v"),
                  _dev(w, torch.float64, ctx.cells, "w"), _dev(p, ctx.pdtype, ctx.cells, "p"))
    if h is not None:
        for c in range(3):
            st.h[c] = _dev(h[c], ctx.pdtype, ctx.comp_numel(c), f"h[{c}]")
    arr, n = _bodies(bodies)
    _ok(_step(ctx.handle, ctypes.byref(st), arr, n, float(dt)), "ibm_step")


def ibm_refine_stats(ctx, reset=False, after_first=False, initial=False):
    """Mixed form: (Poisson solves, FP64-residual corrections, largest final
    max|rhs - L_c phi| * alpha_dt) since the last reset (synchronises); with
    after_first also the largest residual left by the first correction; with
    initial also the largest and the mean residual of the uncorrected solve."""
    out = (c_double * IBM_REFINE_STATS)()
    _ok(_refine_stats(ctx.handle, out, 1 if reset else 0), "ibm_refine_stats")
    r = (int(out[0]), int(out[1]), float(out[2]))
    if after_first:
        r += (float(out[3]),)
    if initial:
        r += (float(out[4]), float(out[5]) / max(1, int(out[0])))
    return r


def ibm_check(ctx):
    f = c_uint32()
    _ok(_check(ctx.handle, ctypes.byref(f)), "ibm_check")
    return int(f.value)


def ibm_profile(ctx, enable=True, filter_=None):
    _ok(_profile(ctx.handle, 1 if enable else 0, filter_.encode() if filter_ else None),
        "ibm_profile")


def ibm_profile_read(ctx, cap=64):
    L = 48
    names = ctypes.create_string_buffer(L * cap)
    cnt = (c_int64 * cap)()
    tot = (c_double * cap)()
    n = _profile_read(ctx.handle, names, L, cnt, tot, cap)
    if n < 0:
        raise IbmError(n, "ibm_profile_read")
    return {names.raw[i * L:(i + 1) * L].split(b"\0")[0].decode(): (int(cnt[i]), float(tot[i]))
            for i in range(n)}


class _Sim:
    """View of one simulation of a batch for the per-context calls
    (ibm_check, tag_lists, ibm_refine_stats)."""

    def __init__(self, handle, nx, ny, nz, pdtype):
        self.handle = handle
        self.cells = nx * ny * nz
        self.vfaces = nx * (ny + 1) * nz
        self.pdtype = pdtype


class Batch:
    """Simulations advanced together on one GPU (include/ibm.h, batch).

    sims: list of dicts with keys nx, ny, nz, lx, lz, y_faces, re, dpdx,
    u, v, w, p (device tensors, kept by pointer), motion ("rigid" or
    "deform"), ref, xyz, vel, tri (device tensors of the body)."""

    def __init__(self, sims, precision="fp64", scheme="rk2", use_q=True, mixed_poisson="fp64",
                 refine_tol=0.0):
        n = len(sims)
        self.n = n
        pdtype = torch.float32 if precision == "mixed" else torch.float64
        grids = (IbmGrid * n)()
        opts = (IbmOpts * n)()
        descs = (IbmSim * n)()
        self._keep = []
        self.shapes = []
        for s, d in enumerate(sims):
            yf = np.ascontiguousarray(np.asarray(d["y_faces"], np.float64))
            self._keep.append(yf)
            nx, ny, nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
            grids[s] = IbmGrid(nx, ny, nz, 0, float(d["lx"]), float(d["lz"]),
                               yf.ctypes.data_as(POINTER(c_double)))
            opts[s] = IbmOpts(IBM_MIXED if precision == "mixed" else IBM_FP64,
                              IBM_RK2CN if scheme == "rk2" else IBM_AB2CN, float(d["re"]),
                              float(d["dpdx"]), 0,
                              IBM_Q_ENERGY if use_q == "energy" else (1 if use_q else 0), 0,
                              float(refine_tol), 1 if mixed_poisson == "refined" else 0, 0)
            cells, vf = nx * ny * nz, nx * (ny + 1) * nz
            st = IbmState(_dev(d["u"], torch.float64, cells, "u"),
                          _dev(d["v"], torch.float64, vf, "v"),
                          _dev(d["w"], torch.float64, cells, "w"),
                          _dev(d["p"], pdtype, cells, "p"))
            deform = d["motion"] == "deform"
            nv = d["xyz"].shape[0]
            nt = d["tri"].shape[0]
            descs[s] = IbmSim(st, MOTION_DEFORM if deform else MOTION_RIGID, nv, nt,
                              _dev(d["ref"], torch.float64, (4 if deform else 3) * nv, "ref"),
                              _dev(d["xyz"], torch.float64, 3 * nv, "xyz"),
                              _dev(d["vel"], torch.float64, 3 * nv, "vel"),
                              _dev(d["tri"], torch.int32, 3 * nt, "tri"))
            self.shapes.append((nx, ny, nz))
        h = c_void_p()
        _ok(_batch_create(grids, opts, descs, n, _stream(), ctypes.byref(h)), "ibm_batch_create")
        self.handle = h
        self.sims = [_Sim(c_void_p(_batch_context(h, s)), *self.shapes[s], pdtype)
                     for s in range(n)]

    def _coef(self, coef):
        cf = np.zeros((self.n, COEF_STRIDE), np.float64)
        for s, c in enumerate(coef):
            c = np.asarray(c, np.float64)
            cf[s, :c.size] = c
        return np.ascontiguousarray(cf)

    def step(self, coef, dt, mode=BATCH_GRAPH):
        cf = self._coef(coef)
        _ok(_batch_step(self.handle, cf.ctypes.data_as(POINTER(c_double)), float(dt), int(mode)),
            "ibm_batch_step")

    @staticmethod
    def _plan_dict(p):
        return {"mode": _MODE_NAMES.get(p.mode, p.mode), "streams": p.streams,
                "rhs_planes": p.rhs_planes, "ms_per_step": p.ms_per_step}

    def tune_scratch_bytes(self):
        nb = int(_batch_tune_bytes(self.handle))
        if nb < 0:
            _ok(nb, "ibm_batch_tune_scratch_bytes")
        return nb

    def tune(self, coef, dt, steps=3, max_entries=64, scratch=None):
        """Autotune the execution plan (ibm_batch_tune, switched off in the
        library: it raises IbmError with IBM_EINVAL); the states are left
        as they were.  scratch: a uint8 device tensor of at least
        tune_scratch_bytes() bytes for the state snapshot (allocated here by
        torch when None; the library allocates nothing).  Returns (best plan,
        list of tried plans), as dicts."""
        cf = self._coef(coef)
        nb = self.tune_scratch_bytes()
        if scratch is None:
            scratch = torch.empty(max(nb, 1), dtype=torch.uint8, device=torch.cuda.current_device())
        ptr = _dev(scratch, torch.uint8, None, "scratch")
        best = IbmBatchPlan()
        table = (IbmBatchPlan * max_entries)()
        ntried = c_int32()
        _ok(_batch_tune(self.handle, cf.ctypes.data_as(POINTER(c_double)), float(dt), int(steps),
                        ptr, scratch.numel(), ctypes.byref(best), table, max_entries,
                        ctypes.byref(ntried)),
            "ibm_batch_tune")
        return self._plan_dict(best), [self._plan_dict(table[k]) for k in range(ntried.value)]

    def set_plan(self, mode="graph", streams=None, rhs_planes=16):
        m = {"graph": BATCH_GRAPH, "streams": BATCH_STREAMS, "grouped": BATCH_GROUPED}[mode]
        p = IbmBatchPlan(m, int(streams or self.n), int(rhs_planes), 0, 0.0)
        _ok(_batch_set_plan(self.handle, ctypes.byref(p)), "ibm_batch_set_plan")

    def get_plan(self):
        p = IbmBatchPlan()
        _ok(_batch_get_plan(self.handle, ctypes.byref(p)), "ibm_batch_get_plan")
        return self._plan_dict(p)

    def check(self):
        f = c_uint32()
        _ok(_batch_check(self.handle, ctypes.byref(f)), "ibm_batch_check")
        return int(f.value)

    def close(self):
        if self.handle:
            _batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
