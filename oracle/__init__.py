"""CPU FP64 oracle of the two-component Shan-Chen D3Q19 lattice Boltzmann
method with moving-boundary ellipsoids (arXiv:1109.3277, Sec. 2).

TEST INFRASTRUCTURE ONLY: this package checks the HIP library. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product package never does, and the two share no code.

The arithmetic lives in ``lb_oracle.c`` (plain loops, FP64, one function per
stage of the method); this module only builds and loads it and marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB = os.path.join(_HERE, "_lb_oracle.so")

# Velocity order of the oracle (rest, 6 axis links, 12 diagonals).
NQ = 19


def _lib_path(plant: int) -> str:
    return _LIB if plant == 0 else os.path.join(_HERE, f"_lb_oracle_plant{plant}.so")


def build(force: bool = True, plant: int = 0) -> str:
    """Compile lb_oracle.c with gcc (FP64, no FMA contraction, OpenMP).
    plant > 0 builds a separate copy with one planted mistake (ORC_PLANT in
    lb_oracle.c), used only by the tests that show a pin catches it."""
    out = _lib_path(plant)
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", f"-DORC_PLANT={int(plant)}", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


_libs = {}


def lib(plant: int = 0):
    L = _libs.get(plant)
    if L is None:
        path = _lib_path(plant)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True, plant=plant)
        L = C.CDLL(path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int]
        L.orc_destroy.argtypes = [P]
        L.orc_init_fields.argtypes = [P, dp, dp, dp]
        L.orc_set_walls.argtypes = [P, C.POINTER(C.c_ubyte), dp]
        L.orc_set_accel.argtypes = [P, dp]
        L.orc_add_ellipsoids.restype = C.c_int
        L.orc_add_ellipsoids.argtypes = [P, C.c_int, dp, dp, dp, dp, dp]
        for name in ("orc_stage_densities", "orc_stage_shell", "orc_stage_collide", "orc_stage_stream",
                     "orc_stage_bodies", "orc_stage_raster_killfill", "orc_stream_only"):
            getattr(L, name).argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int]
        L.orc_sc_force.argtypes = [P, dp, dp]
        L.orc_read_fields.argtypes = [P, dp, dp, dp, ip]
        L.orc_num_particles.restype = C.c_int
        L.orc_num_particles.argtypes = [P]
        L.orc_read_particles.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.orc_read_particle_extra.argtypes = [P, C.c_int, dp]
        L.orc_set_particle_motion.argtypes = [P, C.c_int, dp, dp, dp]
        L.orc_set_particle_accum.argtypes = [P, C.c_int, dp, dp]
        L.orc_stats.argtypes = [P, dp]
        L.orc_step_ledger.argtypes = [P, dp]
        L.orc_get_pops.argtypes = [P, C.c_int, dp]
        L.orc_set_pops.argtypes = [P, C.c_int, dp]
        L.orc_get_rho_internal.argtypes = [P, dp, dp]
        L.orc_set_rho_internal.argtypes = [P, dp, dp]
        L.orc_lattice.argtypes = [ip, ip, ip, dp]
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_read_owner.argtypes = [P, ip]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_pairs.argtypes = [P, C.c_int, C.c_double, C.c_double]
        L.orc_pair_hertz.restype = C.c_double
        L.orc_pair_hertz.argtypes = [P, C.c_int, C.c_int, dp, dp, dp]
        L.orc_pair_lub.argtypes = [P, C.c_int, C.c_int, dp]
        L.orc_set_particle_pose.argtypes = [P, C.c_int, dp, dp]
        _libs[plant] = L
    return L


def _d(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the checker's node loops (timing only; results do not depend on it)."""
    lib().orc_set_threads(int(n))


def lattice():
    """(c [19,3] int, w [19]) in the oracle's velocity order."""
    L = lib()
    cx = (C.c_int * NQ)()
    cy = (C.c_int * NQ)()
    cz = (C.c_int * NQ)()
    w = (C.c_double * NQ)()
    L.orc_lattice(cx, cy, cz, w)
    c = np.stack([np.array(cx[:]), np.array(cy[:]), np.array(cz[:])], axis=1)
    return c, np.array(w[:])


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(NQ)
    uu = _f64(u, 3)
    lib().orc_feq(float(rho), _d(uu), _d(out))
    return out


class Oracle:
    """One periodic nx*ny*nz system (fields indexed [z][y][x], x fastest)."""

    def __init__(self, dims, tau: float, g_br: float, psi_kind: int = 1, plant: int = 0):
        nx, ny, nz = (int(v) for v in dims)
        self.dims = (nx, ny, nz)
        self.N = nx * ny * nz
        self._L = lib(plant)
        self._h = self._L.orc_create(nx, ny, nz, float(tau), float(g_br), int(psi_kind))
        if not self._h:
            raise ValueError("invalid oracle parameters")

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup
    def init_fields(self, rho_a, rho_b, u=None):
        ra = _f64(rho_a, self.N)
        rb = _f64(rho_b, self.N)
        uu = _f64(u, 3 * self.N)
        self._L.orc_init_fields(self._h, _d(ra), _d(rb), _d(uu))

    def set_walls(self, mask, wall_u=None):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        assert m.size == self.N
        wu = _f64(wall_u, 3 * self.N)
        self._L.orc_set_walls(self._h, m.ctypes.data_as(C.POINTER(C.c_ubyte)), _d(wu))

    def set_accel(self, a):
        aa = _f64(a, 3)
        self._L.orc_set_accel(self._h, _d(aa))

    def add_ellipsoids(self, radii, pos, quat, delta_rho=None, density=None):
        radii = _f64(radii)
        n = radii.size // 2
        pos = _f64(pos, 3 * n)
        quat = _f64(quat, 4 * n)
        dr = _f64(delta_rho, n) if delta_rho is not None else None
        de = _f64(density, n) if density is not None else None
        rc = self._L.orc_add_ellipsoids(self._h, n, _d(radii), _d(pos), _d(quat), _d(dr), _d(de))
        if rc != 0:
            raise ValueError(f"orc_add_ellipsoids failed ({rc})")

    # -- stepping
    def step(self, n: int = 1):
        self._L.orc_step(self._h, int(n))

    def stage(self, name: str):
        getattr(self._L, "orc_stage_" + name)(self._h)

    def stream_only(self):
        self._L.orc_stream_only(self._h)

    # -- readout
    def read_fields(self):
        ra = np.zeros(self.N)
        rb = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        own = np.zeros(self.N, dtype=np.int32)
        self._L.orc_read_fields(self._h, _d(ra), _d(rb), _d(u), own.ctypes.data_as(C.POINTER(C.c_int)))
        return ra, rb, u.reshape(-1, 3), own

    def num_particles(self) -> int:
        return self._L.orc_num_particles(self._h)

    def read_particles(self):
        n = self.num_particles()
        out = {k: np.zeros((n, 3)) for k in ("pos", "vel", "omega", "force", "torque")}
        out["quat"] = np.zeros((n, 4))
        self._L.orc_read_particles(self._h, _d(out["pos"]), _d(out["quat"]), _d(out["vel"]),
                                 _d(out["omega"]), _d(out["force"]), _d(out["torque"]))
        return out

    def particle_extra(self, k: int):
        o = np.zeros(20)
        self._L.orc_read_particle_extra(self._h, int(k), _d(o))
        return {"L": o[0:3], "J": o[3:6], "H": o[6:9], "F_links": o[9:12], "T_links": o[12:15],
                "M": o[15], "Iperp": o[16], "Ipar": o[17], "drho": o[18], "dens": o[19]}

    def set_particle_motion(self, k, V=None, L=None, W=None):
        self._L.orc_set_particle_motion(self._h, int(k), _d(_f64(V, 3)), _d(_f64(L, 3)), _d(_f64(W, 3)))

    def set_pairs(self, on=True, K_H=100.0, delta_c=2.0 / 3.0):
        """Particle-particle interactions (Hertz / Berne-Pechukas and lubrication)."""
        self._L.orc_set_pairs(self._h, 1 if on else 0, float(K_H), float(delta_c))

    def pair_hertz(self, i, j):
        """(energy, force on i, torque on i, torque on j) of the Hertz pair term."""
        F, Ti, Tj = np.zeros(3), np.zeros(3), np.zeros(3)
        e = self._L.orc_pair_hertz(self._h, int(i), int(j), _d(F), _d(Ti), _d(Tj))
        return e, F, Ti, Tj

    def pair_lub(self, i, j):
        F = np.zeros(3)
        self._L.orc_pair_lub(self._h, int(i), int(j), _d(F))
        return F

    def set_particle_pose(self, k, X=None, q=None):
        self._L.orc_set_particle_pose(self._h, int(k), _d(_f64(X, 3)), _d(_f64(q, 4)))

    def set_particle_accum(self, k, F, T):
        self._L.orc_set_particle_accum(self._h, int(k), _d(_f64(F, 3)), _d(_f64(T, 3)))

    def stats(self):
        o = np.zeros(8)
        self._L.orc_stats(self._h, _d(o))
        return o

    def ledger(self):
        o = np.zeros(3)
        self._L.orc_step_ledger(self._h, _d(o))
        return {"link_C": o[0], "kill": o[1], "fill": o[2]}

    def get_pops(self, c: int) -> np.ndarray:
        o = np.zeros(NQ * self.N)
        self._L.orc_get_pops(self._h, int(c), _d(o))
        return o.reshape(NQ, self.N)

    def set_pops(self, c: int, f):
        a = _f64(f, NQ * self.N)
        self._L.orc_set_pops(self._h, int(c), _d(a))

    def rho_internal(self):
        ra = np.zeros(self.N)
        rb = np.zeros(self.N)
        self._L.orc_get_rho_internal(self._h, _d(ra), _d(rb))
        return ra, rb

    def set_rho_internal(self, ra, rb):
        self._L.orc_set_rho_internal(self._h, _d(_f64(ra, self.N)), _d(_f64(rb, self.N)))

    def sc_force(self):
        fa = np.zeros(3 * self.N)
        fb = np.zeros(3 * self.N)
        self._L.orc_sc_force(self._h, _d(fa), _d(fb))
        return fa.reshape(-1, 3), fb.reshape(-1, 3)

    def owner(self):
        o = np.zeros(self.N, dtype=np.int32)
        self._L.orc_read_owner(self._h, o.ctypes.data_as(C.POINTER(C.c_int)))
        return o
