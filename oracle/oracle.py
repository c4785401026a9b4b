"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  It never imports the GPU package and the
GPU package never imports it.  See ``picsar_oracle.c`` for the paper sections
each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "picsar_oracle.c")

R_KIND = {"log": 0, "lin": 1}
TH_KIND = {"eqarea": 0, "lin": 1}
MOVER = {"vay": 0, "boris": 1}
BG_KIND = {"none": 0, "uniform_bz": 1, "monopole": 2, "dipole": 3, "dipole_corot": 4}
COMPS = ["Er", "Eth", "Eph", "Br", "Bth", "Bph", "Fr", "Fth", "Fph"]


class _Params(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nth", C.c_int32),
        ("r_in", C.c_double), ("r_out", C.c_double),
        ("r_kind", C.c_int32), ("th_kind", C.c_int32),
        ("c", C.c_double),
        ("n_filt", C.c_int32), ("absorb_cells", C.c_int32),
        ("sigma_max", C.c_double),
        ("mover", C.c_int32), ("bg_kind", C.c_int32),
        ("B0", C.c_double), ("omega", C.c_double), ("t_spin", C.c_double),
        ("q_over_m", C.c_double), ("f_inj", C.c_double), ("q_inj", C.c_double),
        ("inject", C.c_int32), ("seed", C.c_uint64),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE FP64, no fused multiply-add)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.POINTER
        d, i32, i64, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint64
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [P(_Params)]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_error.restype = C.c_char_p
        L.ora_error.argtypes = [C.c_void_p]
        L.ora_field_shape.argtypes = [C.c_void_p, C.c_int, P(i32), P(i32), P(i32)]
        L.ora_set_field.argtypes = [C.c_void_p, C.c_int, P(d)]
        L.ora_get_field.argtypes = [C.c_void_p, C.c_int, P(d)]
        L.ora_add_particles.argtypes = [C.c_void_p, i64] + [P(d)] * 6 + [P(u64)]
        L.ora_add_particles_cells.argtypes = [C.c_void_p, i64, P(i32), P(d), P(i32)] + [P(d)] * 5 + [P(u64)]
        L.ora_num_particles.restype = i64
        L.ora_num_particles.argtypes = [C.c_void_p]
        L.ora_get_particles.argtypes = [C.c_void_p] + [P(d)] * 6 + [P(u64)]
        L.ora_step.argtypes = [C.c_void_p, i32]
        L.ora_step_index.restype = i64
        L.ora_step_index.argtypes = [C.c_void_p]
        L.ora_set_step_index.argtypes = [C.c_void_p, i64]
        L.ora_counters.argtypes = [C.c_void_p, P(i64), P(i64)]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_get_carry.argtypes = [C.c_void_p, P(d)]
        L.ora_set_carry.argtypes = [C.c_void_p, P(d)]
        L.ora_gauss.argtypes = [C.c_void_p, P(d), P(d)]
        L.ora_poynting.argtypes = [C.c_void_p, P(d)]
        L.ora_geometry.argtypes = [C.c_void_p, C.c_int, P(d)]
        L.ora_push_cartesian.argtypes = [C.c_int, P(d), P(d), P(d), d, P(d)]
        L.ora_background.argtypes = [C.c_void_p, d, d, d, P(d), P(d)]
        L.ora_gather.argtypes = [C.c_void_p, d, d, P(d), P(d)]
        L.ora_deposit.argtypes = [C.c_void_p, d, d, d, d, d, d]
        L.ora_clear_F.argtypes = [C.c_void_p]
        L.ora_filter_F.argtypes = [C.c_void_p]
        L.ora_filter_nodes.argtypes = [C.c_void_p, P(d)]
        L.ora_node_charge.argtypes = [C.c_void_p, d, d, d, P(d)]
        L.ora_philox4x64_10.argtypes = [P(u64), P(u64), P(u64)]
        L.ora_ghost.restype = i32
        L.ora_ghost.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().ora_philox4x64_10(_up(c), _up(k), _up(o))
    return o


def push_cartesian(u, E, B, eps, mover="vay"):
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    o = np.zeros(3)
    lib().ora_push_cartesian(MOVER[mover], _dp(u), _dp(E), _dp(B), float(eps), _dp(o))
    return o


class Oracle:
    """One FP64 CPU simulation built from a workload parameter dict."""

    def __init__(self, params: dict):
        p = _Params()
        p.nr, p.nth = int(params["nr"]), int(params["nth"])
        p.r_in, p.r_out = float(params["r_in"]), float(params["r_out"])
        p.r_kind = R_KIND[params.get("r_kind", "log")]
        p.th_kind = TH_KIND[params.get("th_kind", "eqarea")]
        p.c = float(params["c"])
        p.n_filt = int(params.get("n_filt", 0))
        p.absorb_cells = int(params.get("absorb_cells", 0))
        p.sigma_max = float(params.get("sigma_max", 2.0 / max(1, p.absorb_cells)))
        p.mover = MOVER[params.get("mover", "vay")]
        p.bg_kind = BG_KIND[params.get("bg_kind", "none")]
        p.B0 = float(params.get("B0", 0.0))
        p.omega = float(params.get("omega", 0.0))
        p.t_spin = float(params.get("t_spin", 0.0))
        p.q_over_m = float(params.get("q_over_m", 1.0))
        p.f_inj = float(params.get("f_inj", 0.0))
        p.q_inj = float(params.get("q_inj", 1.0))
        p.inject = int(params.get("inject", 0))
        p.seed = int(params.get("seed", 0))
        self.params = dict(params)
        self.p = p
        self._h = lib().ora_create(C.byref(p))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.nr, self.nth = p.nr, p.nth
        self.g = lib().ora_ghost(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ora_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}: {lib().ora_error(self._h).decode()}")

    # fields -------------------------------------------------------------
    def shape(self, comp):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        r, k, r0 = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().ora_field_shape(self._h, c, C.byref(r), C.byref(k), C.byref(r0)))
        return r.value, k.value, r0.value

    def get_field(self, comp):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        r, k, _ = self.shape(c)
        out = np.zeros((r, k))
        self._check(lib().ora_get_field(self._h, c, _dp(out)))
        return out

    def set_field(self, comp, data):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        r, k, _ = self.shape(c)
        a = np.ascontiguousarray(data, dtype=np.float64)
        assert a.shape == (r, k), (a.shape, (r, k))
        self._check(lib().ora_set_field(self._h, c, _dp(a)))

    # particles ------------------------------------------------------------
    def add_particles(self, x, y, ur, ut, up, w, ids=None):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, ur, ut, up, w)]
        n = len(arrs[0])
        idp = None
        if ids is not None:
            ida = np.ascontiguousarray(ids, dtype=np.uint64)
            idp = _up(ida)
        self._check(lib().ora_add_particles(self._h, n, *[_dp(a) for a in arrs], idp))

    def add_particles_cells(self, ci, fx, cj, fy, ur, ut, up, w, ids=None):
        """Particles given as cell indices and in-cell offsets."""
        i32 = [np.ascontiguousarray(a, dtype=np.int32) for a in (ci, cj)]
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (fx, fy, ur, ut, up, w)]
        idp = None
        if ids is not None:
            ida = np.ascontiguousarray(ids, dtype=np.uint64)
            idp = _up(ida)
        ip = [a.ctypes.data_as(C.POINTER(C.c_int32)) for a in i32]
        self._check(lib().ora_add_particles_cells(self._h, len(arrs[0]), ip[0], _dp(arrs[0]), ip[1], _dp(arrs[1]),
                                                  *[_dp(a) for a in arrs[2:]], idp))

    @property
    def n(self):
        return int(lib().ora_num_particles(self._h))

    def particles(self):
        n = self.n
        out = {k: np.zeros(n) for k in ("x", "y", "ur", "ut", "up", "w")}
        ids = np.zeros(n, dtype=np.uint64)
        self._check(lib().ora_get_particles(self._h, *[_dp(out[k]) for k in ("x", "y", "ur", "ut", "up", "w")],
                                            _up(ids)))
        out["id"] = ids
        return out

    # stepping -------------------------------------------------------------
    def step(self, n=1):
        self._check(lib().ora_step(self._h, int(n)))

    @property
    def step_index(self):
        return int(lib().ora_step_index(self._h))

    def set_step_index(self, n):
        lib().ora_set_step_index(self._h, int(n))

    def counters(self):
        a, b = C.c_int64(), C.c_int64()
        lib().ora_counters(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def carry(self):
        out = np.zeros(self.nth + 1)
        lib().ora_get_carry(self._h, _dp(out))
        return out

    def set_carry(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        lib().ora_set_carry(self._h, _dp(a))

    # diagnostics / unit entry points --------------------------------------
    def gauss(self):
        G = np.zeros((self.nr + 1, self.nth + 1))
        Q = np.zeros_like(G)
        self._check(lib().ora_gauss(self._h, _dp(G), _dp(Q)))
        return G, Q

    def luminosity(self):
        """Poynting luminosity through the sphere of each radial half-node."""
        out = np.zeros(self.nr)
        self._check(lib().ora_poynting(self._h, _dp(out)))
        return out

    def geometry(self, which):
        sizes = {0: self.nr + 1, 1: self.nr, 2: self.nth + 1, 3: self.nth + 1, 4: self.nth + 1,
                 5: (self.nr + 1) * (self.nth + 1)}
        out = np.zeros(sizes[which])
        self._check(lib().ora_geometry(self._h, which, _dp(out)))
        if which == 5:
            out = out.reshape(self.nr + 1, self.nth + 1)
        return out

    def background(self, x, y, t):
        E, B = np.zeros(3), np.zeros(3)
        lib().ora_background(self._h, float(x), float(y), float(t), _dp(E), _dp(B))
        return E, B

    def gather(self, x, y):
        E, B = np.zeros(3), np.zeros(3)
        lib().ora_gather(self._h, float(x), float(y), _dp(E), _dp(B))
        return E, B

    def deposit(self, x0, y0, x1, y1, Q, dphi=0.0):
        self._check(lib().ora_deposit(self._h, x0, y0, x1, y1, Q, dphi))

    def clear_F(self):
        lib().ora_clear_F(self._h)

    def filter_F(self):
        self._check(lib().ora_filter_F(self._h))

    def filter_nodes(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        self._check(lib().ora_filter_nodes(self._h, _dp(rho)))
        return rho

    def node_charge(self, x, y, Q, rho=None):
        if rho is None:
            rho = np.zeros((self.nr + 1 + 2 * self.g, self.nth + 1))
        self._check(lib().ora_node_charge(self._h, float(x), float(y), float(Q), _dp(rho)))
        return rho
