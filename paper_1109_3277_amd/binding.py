"""ctypes binding of liblbe's C ABI (include/lbe.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies the device workspace and the stream. Importing this module
on a machine without the built library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbe.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_EUNSTABLE, LB_ESTATE, LB_EGEOM = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16_dev": 2, "bf16_dev": 3}
EXPORTED = [
    "lb_workspace_bytes", "lb_create", "lb_destroy", "lb_init_fields", "lb_add_ellipsoids", "lb_step",
    "lb_step_async", "lb_read_fields", "lb_read_fields_dev", "lb_num_particles", "lb_read_particles", "lb_set_particle_motion", "lb_stats",
    "lb_set_body_accel", "lb_set_static_solid", "lb_set_pair_interactions", "lb_state_bytes", "lb_save_state", "lb_load_state", "lb_last_error",
    "lb_profile_enable", "lb_profile_read", "lb_batch_workspace_bytes", "lb_create_batch", "lb_init_fields_sys",
    "lb_add_ellipsoids_sys", "lb_read_fields_sys", "lb_read_particles_sys", "lb_stats_sys", "lb_batch_size",
    "lb_batch_system", "lb_batch_tune", "lb_batch_last_graph", "lb_stats_noalloc", "lb_domain_size",
]
PHASES = ["density", "shell", "fused", "forces", "bodies", "raster", "killfill"]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbe error {code}: {msg}")
        self.code = code


class lb_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double),
                ("g_br", C.c_double), ("psi_kind", C.c_int32), ("precision", C.c_int32),
                ("max_particles", C.c_int32), ("max_radius", C.c_double)]


TUNE_CANDIDATES = 3


class lb_tune_result(C.Structure):
    _fields_ = [("tile_width", C.c_int32), ("cached", C.c_int32), ("tile_widths", C.c_int32 * TUNE_CANDIDATES),
                ("ms", C.c_double * TUNE_CANDIDATES)]


_lib = None


def load_library():
    """Load liblbe.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run python -m paper_1109_3277_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    pp = C.POINTER(lb_params)
    L.lb_workspace_bytes.restype = C.c_size_t
    L.lb_workspace_bytes.argtypes = [pp]
    L.lb_create.argtypes = [pp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lb_destroy.argtypes = [vp]
    L.lb_destroy.restype = None
    L.lb_init_fields.argtypes = [vp, dp, dp, dp]
    L.lb_add_ellipsoids.argtypes = [vp, C.c_int32, dp, dp, dp, dp, dp]
    L.lb_step.argtypes = [vp, C.c_int32]
    L.lb_step_async.argtypes = [vp, C.c_int32]
    L.lb_read_fields.argtypes = [vp, dp, dp, dp, ip]
    L.lb_read_fields_dev.argtypes = [vp, vp, vp, vp, vp]
    L.lb_num_particles.argtypes = [vp]
    L.lb_read_particles.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    L.lb_set_particle_motion.argtypes = [vp, C.c_int32, dp, dp, dp]
    L.lb_stats.argtypes = [vp, dp]
    L.lb_set_body_accel.argtypes = [vp, dp]
    L.lb_set_static_solid.argtypes = [vp, C.POINTER(C.c_uint8), dp]
    L.lb_set_pair_interactions.argtypes = [vp, C.c_int, C.c_double, C.c_double]
    L.lb_state_bytes.restype = C.c_size_t
    L.lb_state_bytes.argtypes = [vp]
    L.lb_save_state.argtypes = [vp, vp, C.c_size_t]
    L.lb_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lb_last_error.restype = C.c_char_p
    L.lb_last_error.argtypes = [vp]
    L.lb_profile_enable.argtypes = [vp, C.c_int]
    L.lb_profile_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.lb_batch_workspace_bytes.restype = C.c_size_t
    L.lb_batch_workspace_bytes.argtypes = [C.c_int32, pp]
    L.lb_create_batch.argtypes = [C.c_int32, pp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lb_init_fields_sys.argtypes = [vp, C.c_int32, dp, dp, dp]
    L.lb_add_ellipsoids_sys.argtypes = [vp, C.c_int32, C.c_int32, dp, dp, dp, dp, dp]
    L.lb_read_fields_sys.argtypes = [vp, C.c_int32, dp, dp, dp, ip]
    L.lb_read_particles_sys.argtypes = [vp, C.c_int32, dp, dp, dp, dp, dp, dp]
    L.lb_stats_sys.argtypes = [vp, C.c_int32, dp]
    L.lb_batch_size.argtypes = [vp]
    L.lb_batch_system.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    L.lb_batch_tune.argtypes = [vp, C.POINTER(lb_tune_result)]
    L.lb_batch_last_graph.argtypes = [vp, ip, C.POINTER(C.c_int64)]
    L.lb_stats_noalloc.argtypes = [vp, vp]
    L.lb_domain_size.argtypes = [vp, dp]
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_params(dims, tau, g_br, psi_kind=1, precision="fp64", max_particles=0, max_radius=0.0) -> lb_params:
    nx, ny, nz = (int(v) for v in dims)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return lb_params(nx, ny, nz, float(tau), float(g_br), int(psi_kind), prec, int(max_particles), float(max_radius))


def workspace_bytes(params: lb_params) -> int:
    return int(load_library().lb_workspace_bytes(C.byref(params)))


class Lattice:
    """One periodic two-component system on the GPU (fields [z][y][x])."""

    def __init__(self, dims, tau, g_br, psi_kind=1, precision="fp64", max_particles=0, max_radius=0.0,
                 device="cuda", _borrowed=None):
        import torch

        L = load_library()
        if _borrowed is not None:  # a system of a Batch: handle owned by the batch
            owner, h, params = _borrowed
            self._batch, self._h, self.params = owner, h, params
            self.dims = (params.nx, params.ny, params.nz)
            self.N = params.nx * params.ny * params.nz
            self._borrowed = True
            return
        self._borrowed = False
        self.params = make_params(dims, tau, g_br, psi_kind, precision, max_particles, max_radius)
        self.dims = tuple(int(v) for v in dims)
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        nbytes = L.lb_workspace_bytes(C.byref(self.params))
        if nbytes == 0:
            raise LBError(LB_EINVAL, "invalid parameters")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self._ws.device)
        h = C.c_void_p()
        rc = L.lb_create(C.byref(self.params), C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                         C.byref(h))
        if rc != 0:
            raise LBError(rc, L.lb_last_error(None).decode())
        self._h = h

    # -- plumbing
    def _check(self, rc):
        if rc != 0:
            raise LBError(rc, load_library().lb_last_error(self._h).decode())

    def close(self):
        """Destroy the handle and drop the workspace tensor (the memory goes
        back to torch's allocator)."""
        if getattr(self, "_h", None) and not getattr(self, "_borrowed", False):
            load_library().lb_destroy(self._h)
        self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- API
    def init_fields(self, rho_a, rho_b, u=None):
        ra, rb = _f64(rho_a, self.N), _f64(rho_b, self.N)
        uu = _f64(u, 3 * self.N)
        self._check(load_library().lb_init_fields(self._h, _dp(ra), _dp(rb), _dp(uu)))

    def add_ellipsoids(self, radii, pos, quat, delta_rho=None, density=None):
        radii = _f64(radii)
        n = radii.size // 2
        pos, quat = _f64(pos, 3 * n), _f64(quat, 4 * n)
        dr = _f64(delta_rho, n)
        de = _f64(density, n)
        self._check(load_library().lb_add_ellipsoids(self._h, n, _dp(radii), _dp(pos), _dp(quat), _dp(dr), _dp(de)))

    def step(self, n=1):
        self._check(load_library().lb_step(self._h, int(n)))

    def step_async(self, n=1):
        self._check(load_library().lb_step_async(self._h, int(n)))

    def set_body_accel(self, a):
        aa = _f64(a, 3)
        self._check(load_library().lb_set_body_accel(self._h, _dp(aa)))

    def set_pair_interactions(self, on=True, K_H=100.0, delta_c=2.0 / 3.0):
        """Hertz / Berne-Pechukas repulsion and lubrication between particles."""
        self._check(load_library().lb_set_pair_interactions(self._h, 1 if on else 0, float(K_H), float(delta_c)))

    def set_static_solid(self, mask, wall_u=None):
        """Wall nodes (mask, N entries, x fastest) with one velocity wall_u
        (3 values, None for resting walls); before init_fields."""
        m = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
        if m.size != self.N:
            raise ValueError("mask needs one entry per node")
        wu = None if wall_u is None else _f64(wall_u, 3)
        self._check(load_library().lb_set_static_solid(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                     None if wu is None else _dp(wu)))

    def read_fields(self):
        ra, rb, u = np.zeros(self.N), np.zeros(self.N), np.zeros(3 * self.N)
        own = np.zeros(self.N, dtype=np.int32)
        self._check(load_library().lb_read_fields(self._h, _dp(ra), _dp(rb), _dp(u),
                                                  own.ctypes.data_as(C.POINTER(C.c_int32))))
        return ra, rb, u.reshape(-1, 3), own

    def read_fields_dev(self, rho_a=None, rho_b=None, u=None, owner=None):
        """Fields into torch device tensors (float64 N, N, N x 3; int32 N; any
        may be None), ordered on the handle's stream."""
        def ptr(t, dtype, n):
            if t is None:
                return None
            import torch
            assert t.is_cuda and t.dtype == dtype and t.numel() == n and t.is_contiguous()
            return C.c_void_p(t.data_ptr())
        import torch
        self._check(load_library().lb_read_fields_dev(
            self._h, ptr(rho_a, torch.float64, self.N), ptr(rho_b, torch.float64, self.N),
            ptr(u, torch.float64, 3 * self.N), ptr(owner, torch.int32, self.N)))

    def num_particles(self) -> int:
        return int(load_library().lb_num_particles(self._h))

    def read_particles(self):
        n = self.num_particles()
        out = {k: np.zeros((n, 3)) for k in ("pos", "vel", "omega", "force", "torque")}
        out["quat"] = np.zeros((n, 4))
        self._check(load_library().lb_read_particles(self._h, _dp(out["pos"]), _dp(out["quat"]), _dp(out["vel"]),
                                                     _dp(out["omega"]), _dp(out["force"]), _dp(out["torque"])))
        return out

    def set_particle_motion(self, k, vel=None, omega=None, angmom=None):
        """Velocity, angular velocity and angular momentum (space frame) of
        particle k; None leaves that quantity as it is."""
        args = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(3) for a in (vel, omega, angmom)]
        self._check(load_library().lb_set_particle_motion(self._h, int(k), *[_dp(a) for a in args]))

    def stats(self):
        o = np.zeros(8)
        self._check(load_library().lb_stats(self._h, _dp(o)))
        return o

    def domain_size(self):
        """Eq. (12): [L_x, L_y, L_z, L, <k_x^2>, <k_y^2>, <k_z^2>, sum_k S(k)]."""
        o = np.zeros(8)
        self._check(load_library().lb_domain_size(self._h, _dp(o)))
        return o

    def profile(self, on: bool):
        self._check(load_library().lb_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{phase: (total ms, launches)} of the launches recorded since profile(True)."""
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), dtype=np.int64)
        self._check(load_library().lb_profile_read(self._h, _dp(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64))))
        return {p: (float(ms[k]), int(cnt[k])) for k, p in enumerate(PHASES)}

    def save_state(self) -> bytes:
        L = load_library()
        n = L.lb_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        self._check(L.lb_save_state(self._h, buf, n))
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(load_library().lb_load_state(self._h, buf, len(data)))


class Batch:
    """Independent periodic systems advanced together (one launch per phase
    over all systems, steps replayed as a HIP graph). `params` is a list of
    dicts with the Lattice arguments dims, tau, g_br and optionally psi_kind,
    max_particles, max_radius; all systems share `precision`."""

    def __init__(self, params, precision="fp64", device="cuda"):
        import torch

        L = load_library()
        plist = [make_params(p["dims"], p["tau"], p["g_br"], p.get("psi_kind", 1), precision,
                             p.get("max_particles", 0), p.get("max_radius", 0.0)) for p in params]
        arr = (lb_params * len(plist))(*plist)
        nbytes = L.lb_batch_workspace_bytes(len(plist), arr)
        if nbytes == 0:
            raise LBError(LB_EINVAL, "invalid batch parameters")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self._ws.device)
        h = C.c_void_p()
        rc = L.lb_create_batch(len(plist), arr, C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                               C.byref(h))
        if rc != 0:
            raise LBError(rc, L.lb_last_error(None).decode())
        self._h = h
        self.systems = []
        for k, prm in enumerate(plist):
            sh = C.c_void_p()
            self._check(L.lb_batch_system(self._h, k, C.byref(sh)))
            self.systems.append(Lattice(None, None, None, _borrowed=(self, sh, prm)))

    def _check(self, rc):
        if rc != 0:
            raise LBError(rc, load_library().lb_last_error(self._h).decode())

    def __len__(self):
        return len(self.systems)

    def __getitem__(self, k) -> Lattice:
        return self.systems[k]

    def step(self, n=1):
        self._check(load_library().lb_step(self._h, int(n)))

    def step_async(self, n=1):
        self._check(load_library().lb_step_async(self._h, int(n)))

    def tune(self) -> int:
        """Autotune the fused tile shape; returns the chosen tile width."""
        return self.tune_report()["tile_width"]

    def tune_report(self) -> dict:
        r = lb_tune_result()
        self._check(load_library().lb_batch_tune(self._h, C.byref(r)))
        cand = {f"{w}x{256 // w}": round(float(m), 5) for w, m in zip(r.tile_widths, r.ms)}
        return {"tile_width": int(r.tile_width), "tile": f"{r.tile_width}x{256 // r.tile_width}",
                "cached": bool(r.cached), "candidates": cand, "best_ms": float(min(r.ms))}

    def last_graph(self):
        """(steps, kernel nodes) of the graph the last step call launched."""
        st, nodes = C.c_int32(0), C.c_int64(0)
        self._check(load_library().lb_batch_last_graph(self._h, C.byref(st), C.byref(nodes)))
        return int(st.value), int(nodes.value)

    def close(self):
        for s in getattr(self, "systems", []):
            s._h = None
        if getattr(self, "_h", None):
            load_library().lb_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
