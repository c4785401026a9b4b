"""ctypes binding of libpicsar_hip.so (the C ABI in include/picsar_hip.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpicsar_hip.so")

R_KIND = {"log": 0, "lin": 1}
TH_KIND = {"eqarea": 0, "lin": 1}
PRECISION = {"fp64": 0, "fp32": 1}
MOVER = {"vay": 0, "boris": 1}
BG_KIND = {"none": 0, "uniform_bz": 1, "monopole": 2, "dipole": 3, "dipole_corot": 4}
COMPS = ["Er", "Eth", "Eph", "Br", "Bth", "Bph", "Fr", "Fth", "Fph"]
FLAG_IDS = 1
MOM_COUNTS, MOM_GAUSS, MOM_CARRY, MOM_STAGE_MS, MOM_POYNTING, MOM_GAUSS_RES, MOM_RHO_Q = 0, 1, 2, 3, 4, 5, 6
GAUSS_RES_KEYS = ["drift_max", "drift_l2", "res_max", "res_l2", "abs_charge_max", "flux_max", "nodes", "non_finite",
                  "ref_step"]
STAGES = ["sort", "faraday", "push", "filter", "ampere", "absorb", "inject", "zero", "total"]

# (tile_r, tile_th, sort interval) tried by Sim.autotune by default
AUTOTUNE_CANDIDATES = [(4, 8, 4), (4, 8, 8), (8, 8, 8), (4, 4, 4), (8, 16, 8), (4, 8, 16)]

STATUS = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_ECFL", -4: "PIC_ECAPACITY",
          -5: "PIC_ENAN", -6: "PIC_EDEVICE", -7: "PIC_ESTATE"}

EXPORTED = ["pic_create", "pic_init", "pic_init_grid", "pic_inject_particles", "pic_inject_particles_noalloc", "pic_step", "pic_field_shape", "pic_get_field",
            "pic_set_field", "pic_get_particles", "pic_get_particle_cells", "pic_get_moments", "pic_set_step_index", "pic_set_carry",
            "pic_set_timing", "pic_set_sort", "pic_autotune", "pic_save", "pic_load", "pic_last_error", "pic_destroy",
            "pic_batch_create", "pic_batch_step", "pic_batch_elapsed_ms", "pic_batch_set_timing",
            "pic_batch_stage_ms", "pic_batch_last_error", "pic_batch_destroy"]


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nth", C.c_int32), ("r_in", C.c_double), ("r_out", C.c_double),
                ("r_kind", C.c_int32), ("th_kind", C.c_int32), ("c", C.c_double), ("n_filt", C.c_int32),
                ("absorb_cells", C.c_int32), ("sigma_max", C.c_double), ("precision", C.c_int32),
                ("mover", C.c_int32), ("particle_capacity", C.c_int64), ("tile_r", C.c_int32),
                ("tile_th", C.c_int32), ("sort_interval", C.c_int32), ("flags", C.c_int32),
                ("chunk_ppt", C.c_int32)]


class PhysDesc(C.Structure):
    _fields_ = [("bg_kind", C.c_int32), ("B0", C.c_double), ("omega", C.c_double), ("t_spin", C.c_double),
                ("q_over_m", C.c_double), ("f_inj", C.c_double), ("q_inj", C.c_double), ("inject", C.c_int32),
                ("seed", C.c_uint64)]


_lib = None


def lib():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run paper_1407_1810_amd/build.py")
        L = C.CDLL(LIB)
        P, d, i32, i64, u64, vp = C.POINTER, C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
        L.pic_create.argtypes = [P(vp), C.c_int, vp]
        L.pic_init.argtypes = [vp, P(GridDesc), P(PhysDesc)]
        L.pic_init_grid.argtypes = [vp, P(GridDesc), P(PhysDesc)]
        L.pic_inject_particles.argtypes = [vp, i64] + [P(d)] * 6 + [P(u64)]
        L.pic_inject_particles_noalloc.argtypes = [vp, i64] + [P(d)] * 6 + [P(u64)]
        L.pic_step.argtypes = [vp, i32]
        L.pic_field_shape.argtypes = [vp, i32, P(i32), P(i32), P(i32)]
        L.pic_get_field.argtypes = [vp, i32, P(d), i64]
        L.pic_set_field.argtypes = [vp, i32, P(d), i64]
        L.pic_get_particles.argtypes = [vp] + [P(d)] * 6 + [P(u64), i64, P(i64)]
        L.pic_get_particle_cells.argtypes = [vp, P(i32), P(i32), P(d), P(d), i64, P(i64)]
        L.pic_get_moments.argtypes = [vp, i32, P(d), i64]
        L.pic_set_step_index.argtypes = [vp, i64]
        L.pic_set_carry.argtypes = [vp, P(d), i64]
        L.pic_set_timing.argtypes = [vp, i32]
        L.pic_set_sort.argtypes = [vp, i32, i32, i32]
        L.pic_autotune.argtypes = [vp, P(i32), i32, i32, P(i32), P(d)]
        L.pic_save.argtypes = [vp, C.c_char_p]
        L.pic_load.argtypes = [vp, C.c_char_p]
        L.pic_last_error.argtypes = [vp]
        L.pic_last_error.restype = C.c_char_p
        L.pic_destroy.argtypes = [vp]
        L.pic_batch_create.argtypes = [P(vp), i32, vp, P(vp)]
        L.pic_batch_step.argtypes = [vp, i32]
        L.pic_batch_elapsed_ms.argtypes = [vp, P(d)]
        L.pic_batch_set_timing.argtypes = [vp, i32]
        L.pic_batch_stage_ms.argtypes = [vp, P(d), i64]
        L.pic_batch_last_error.argtypes = [vp]
        L.pic_batch_last_error.restype = C.c_char_p
        L.pic_batch_destroy.argtypes = [vp]
        for name in ("pic_create", "pic_init", "pic_init_grid", "pic_inject_particles", "pic_inject_particles_noalloc", "pic_step", "pic_field_shape",
                     "pic_get_field", "pic_set_field", "pic_get_particles", "pic_get_particle_cells",
                     "pic_get_moments",
                     "pic_set_step_index", "pic_set_carry", "pic_set_timing", "pic_set_sort", "pic_autotune",
                     "pic_batch_create",
                     "pic_batch_step", "pic_batch_elapsed_ms", "pic_batch_set_timing", "pic_batch_stage_ms"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint64))


class Sim:
    """One GPU simulation.  `params` is a workload parameter dict (grid,
    numerics and analytic-field keys, see workloads.py)."""

    def __init__(self, params: dict, precision: str = "fp64", capacity: int = 1 << 20, device: int = 0,
                 tile=(0, 0), sort_interval: int = 0, ids: bool = True, stream=None, chunk_ppt: int = 0):
        L = lib()
        self._h = C.c_void_p()
        rc = L.pic_create(C.byref(self._h), int(device), stream)
        if rc != 0:
            raise PicError(rc, "pic_create failed (no HIP device?)")
        g = GridDesc()
        g.nr, g.nth = int(params["nr"]), int(params["nth"])
        g.r_in, g.r_out = float(params["r_in"]), float(params["r_out"])
        g.r_kind = R_KIND[params.get("r_kind", "log")]
        g.th_kind = TH_KIND[params.get("th_kind", "eqarea")]
        g.c = float(params["c"])
        g.n_filt = int(params.get("n_filt", 0))
        g.absorb_cells = int(params.get("absorb_cells", 0))
        g.sigma_max = float(params.get("sigma_max", 2.0 / max(1, g.absorb_cells)))
        g.precision = PRECISION[precision]
        g.mover = MOVER[params.get("mover", "vay")]
        g.particle_capacity = int(capacity)
        g.tile_r, g.tile_th = int(tile[0]), int(tile[1])
        g.sort_interval = int(sort_interval)
        g.flags = FLAG_IDS if ids else 0
        g.chunk_ppt = int(chunk_ppt)
        ph = PhysDesc()
        ph.bg_kind = BG_KIND[params.get("bg_kind", "none")]
        ph.B0 = float(params.get("B0", 0.0))
        ph.omega = float(params.get("omega", 0.0))
        ph.t_spin = float(params.get("t_spin", 0.0))
        ph.q_over_m = float(params.get("q_over_m", 1.0))
        ph.f_inj = float(params.get("f_inj", 0.0))
        ph.q_inj = float(params.get("q_inj", 1.0))
        ph.inject = int(params.get("inject", 0))
        ph.seed = int(params.get("seed", 0))
        self.grid, self.phys = g, ph
        self.nr, self.nth = g.nr, g.nth
        self.precision = precision
        self._check(L.pic_init_grid(self._h, C.byref(g), C.byref(ph)))

    @classmethod
    def load(cls, path, device: int = 0, stream=None):
        """A simulation restored from a checkpoint written by save(): the
        same grid, physics, sort settings and state, continuing the run."""
        self = cls.__new__(cls)
        L = lib()
        self._h = C.c_void_p()
        rc = L.pic_create(C.byref(self._h), int(device), stream)
        if rc != 0:
            raise PicError(rc, "pic_create failed (no HIP device?)")
        try:
            self._check(L.pic_load(self._h, os.fsencode(os.fspath(path))))
            rows, cols, row0 = C.c_int32(), C.c_int32(), C.c_int32()
            self._check(L.pic_field_shape(self._h, COMPS.index("Eph"), C.byref(rows), C.byref(cols), C.byref(row0)))
        except Exception:
            self.close()
            raise
        self.grid = self.phys = self.precision = None
        self.nr, self.nth = rows.value - 1, cols.value - 1
        return self

    def save(self, path):
        """Checkpoint the whole state to `path` (see pic_save)."""
        self._check(lib().pic_save(self._h, os.fsencode(os.fspath(path))))

    def _check(self, rc):
        if rc != 0:
            raise PicError(rc, lib().pic_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pic_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # particles --------------------------------------------------------------
    def add_particles(self, x, y, ur, ut, up, w, ids=None):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, ur, ut, up, w)]
        idp = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint64)
        self._check(lib().pic_inject_particles(self._h, len(a[0]), *[_dp(v) for v in a], _up(idp)))

    def add_particles_noalloc(self, x, y, ur, ut, up, w, ids=None):
        """add_particles through pic_inject_particles_noalloc (no device
        allocation; at most 65536 particles per call)."""
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, ur, ut, up, w)]
        idp = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint64)
        self._check(lib().pic_inject_particles_noalloc(self._h, len(a[0]), *[_dp(v) for v in a], _up(idp)))

    def particles(self):
        n = int(self.counts()["live"])
        out = {k: np.zeros(n) for k in ("x", "y", "ur", "ut", "up", "w")}
        ids = np.zeros(n, dtype=np.uint64)
        got = C.c_int64()
        self._check(lib().pic_get_particles(self._h, *[_dp(out[k]) for k in ("x", "y", "ur", "ut", "up", "w")],
                                            _up(ids), n, C.byref(got)))
        out["id"] = ids
        return out

    def particle_cells(self):
        """Cell indices and in-cell offsets of the live particles, exactly as
        stored, in the order of particles()."""
        n = int(self.counts()["live"])
        ci, cj = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
        fx, fy = np.zeros(n), np.zeros(n)
        got = C.c_int64()
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        self._check(lib().pic_get_particle_cells(self._h, ip(ci), ip(cj), _dp(fx), _dp(fy), n, C.byref(got)))
        return dict(ci=ci, cj=cj, fx=fx, fy=fy)

    # stepping ----------------------------------------------------------------
    def step(self, n=1):
        self._check(lib().pic_step(self._h, int(n)))

    def set_step_index(self, n):
        self._check(lib().pic_set_step_index(self._h, int(n)))

    def set_timing(self, on=True):
        self._check(lib().pic_set_timing(self._h, 1 if on else 0))

    def set_sort(self, tile_r, tile_th, sort_interval):
        self._check(lib().pic_set_sort(self._h, int(tile_r), int(tile_th), int(sort_interval)))

    def autotune(self, candidates=None, steps=8):
        """Pick the sort tile and interval with the least device time per
        particle-step among `candidates` ((tile_r, tile_th, interval) tuples);
        the tuning steps advance the run.  Returns (best, ns per particle-step)."""
        cands = AUTOTUNE_CANDIDATES if candidates is None else [tuple(int(v) for v in c) for c in candidates]
        flat = np.ascontiguousarray(np.array(cands, dtype=np.int32).reshape(-1))
        best = np.zeros(3, dtype=np.int32)
        ns = C.c_double()
        self._check(lib().pic_autotune(self._h, flat.ctypes.data_as(C.POINTER(C.c_int32)), len(cands), int(steps),
                                       best.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(ns)))
        return tuple(int(v) for v in best), ns.value

    # fields ------------------------------------------------------------------
    def shape(self, comp):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        r, k, r0 = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().pic_field_shape(self._h, c, C.byref(r), C.byref(k), C.byref(r0)))
        return r.value, k.value, r0.value

    def get_field(self, comp):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        r, k, _ = self.shape(c)
        out = np.zeros((r, k))
        self._check(lib().pic_get_field(self._h, c, _dp(out), out.size))
        return out

    def set_field(self, comp, data):
        c = COMPS.index(comp) if isinstance(comp, str) else int(comp)
        a = np.ascontiguousarray(data, dtype=np.float64)
        self._check(lib().pic_set_field(self._h, c, _dp(a), a.size))

    # moments -----------------------------------------------------------------
    def counts(self):
        out = np.zeros(6)
        self._check(lib().pic_get_moments(self._h, MOM_COUNTS, _dp(out), 6))
        return dict(live=int(out[0]), injected=int(out[1]), deleted=int(out[2]), step=int(out[3]),
                    particle_steps=int(out[4]), global_chunks=int(out[5]))

    def gauss(self):
        N = (self.nr + 1) * (self.nth + 1)
        out = np.zeros(2 * N)
        self._check(lib().pic_get_moments(self._h, MOM_GAUSS, _dp(out), out.size))
        return out[:N].reshape(self.nr + 1, self.nth + 1), out[N:].reshape(self.nr + 1, self.nth + 1)

    def gauss_residual(self):
        """The Gauss residual R = G - Qbar reduced on the device in FP64 over
        the interior nodes (PIC_MOM_GAUSS_RES): a dict of GAUSS_RES_KEYS.  The
        drift is against the residual of the first Gauss evaluation since the
        state was last set from the host."""
        out = np.zeros(len(GAUSS_RES_KEYS))
        self._check(lib().pic_get_moments(self._h, MOM_GAUSS_RES, _dp(out), out.size))
        return dict(zip(GAUSS_RES_KEYS, out.tolist()))

    def rho_q(self):
        """The filtered bilinear node charge Qbar, (nr + 1) x (nth + 1)."""
        out = np.zeros((self.nr + 1, self.nth + 1))
        self._check(lib().pic_get_moments(self._h, MOM_RHO_Q, _dp(out), out.size))
        return out

    def luminosity(self):
        """Poynting luminosity (total field) through the sphere of each
        radial half-node, computed on the device in FP64."""
        out = np.zeros(self.nr)
        self._check(lib().pic_get_moments(self._h, MOM_POYNTING, _dp(out), out.size))
        return out

    def carry(self):
        out = np.zeros(self.nth + 1)
        self._check(lib().pic_get_moments(self._h, MOM_CARRY, _dp(out), out.size))
        return out

    def set_carry(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._check(lib().pic_set_carry(self._h, _dp(a), a.size))

    def stage_ms(self):
        out = np.zeros(9)
        self._check(lib().pic_get_moments(self._h, MOM_STAGE_MS, _dp(out), 9))
        return dict(zip(STAGES, out.tolist()))


class Batch:
    """Several Sim objects (same precision, same device) stepped together by
    one launch sequence per step (pic_batch_*).  The Sims stay usable for
    reading fields, particles and counts; keep them alive while the batch
    exists."""

    def __init__(self, sims, stream=None):
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        self._h = C.c_void_p()
        rc = lib().pic_batch_create(arr, len(self.sims), stream, C.byref(self._h))
        if rc != 0:
            raise PicError(rc, "pic_batch_create failed")

    def _check(self, rc):
        if rc != 0:
            raise PicError(rc, lib().pic_batch_last_error(self._h).decode())

    def step(self, n=1):
        self._check(lib().pic_batch_step(self._h, int(n)))

    def elapsed_ms(self):
        out = C.c_double()
        self._check(lib().pic_batch_elapsed_ms(self._h, C.byref(out)))
        return out.value

    def set_timing(self, on=True):
        self._check(lib().pic_batch_set_timing(self._h, 1 if on else 0))

    def stage_ms(self):
        out = np.zeros(9)
        self._check(lib().pic_batch_stage_ms(self._h, _dp(out), 9))
        return dict(zip(STAGES, out.tolist()))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pic_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gpu_available() -> bool:
    """True if a HIP device is visible (used to skip GPU tests on CPU hosts)."""
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False
