"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  It never imports the GPU package and the GPU package never imports
it.  Instance descriptors are the plain dicts written by the shared input
generators.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Species(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("w0", C.c_double), ("mcc", C.c_int),
                ("sigma_el", C.c_double), ("sigma_iz", C.c_double), ("eps_iz", C.c_double),
                ("sigma_cx", C.c_double), ("eps_max", C.c_double)]


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("precision", C.c_int), ("length", C.c_double), ("dt", C.c_double),
                ("ncells", C.c_int), ("min_level", C.c_int), ("max_level", C.c_int), ("base_level", C.c_int),
                ("refine_disk", C.c_int), ("disk_cx", C.c_double), ("disk_cy", C.c_double),
                ("disk_r", C.c_double), ("disk_level", C.c_int), ("field_bc", C.c_int * 4),
                ("wall_phi", C.c_double * 4), ("particle_bc", C.c_int), ("depth_z", C.c_double),
                ("gas_density", C.c_double), ("gas_temperature", C.c_double), ("gas_mass", C.c_double),
                ("seed", C.c_uint64), ("instance_key", C.c_uint32), ("nspecies", C.c_int),
                ("species", Species * 2), ("field_scheme", C.c_int),
                ("leaf_keys", C.c_void_p), ("leaf_levels", C.c_void_p), ("nleaves", C.c_int64),
                ("disk_cz", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("alive_start", C.c_int64 * 2), ("absorbed", C.c_int64 * 2), ("elastic", C.c_int64),
                ("ionization", C.c_int64), ("cx", C.c_int64), ("births", C.c_int64),
                ("numax_violations", C.c_int64 * 2), ("lost_reflect", C.c_int64)]

    def as_dict(self):
        return dict(alive_start=list(self.alive_start), absorbed=list(self.absorbed), elastic=self.elastic,
                    ionization=self.ionization, cx=self.cx, births=self.births,
                    numax_violations=list(self.numax_violations), lost_reflect=self.lost_reflect)


class AdaptStats(C.Structure):
    _fields_ = [("refined", C.c_int64), ("coarsened", C.c_int64), ("balance_refined", C.c_int64),
                ("split_parents", C.c_int64), ("merged_pairs", C.c_int64), ("nleaves", C.c_int64),
                ("merge_energy_change", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "oracle.cpp")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        _LIB = load_lib(path)
    return _LIB


def load_lib(path):
    """Load an oracle shared library at 'path' and declare its functions."""
    L = C.CDLL(path)
    P = C.c_void_p
    L.or_create.restype = P
    L.or_create.argtypes = [C.POINTER(Desc)]
    L.or_destroy.argtypes = [P]
    L.or_load.argtypes = [P, C.c_int, C.c_int64, P, P, P, P]
    L.or_count.restype = C.c_int64
    L.or_count.argtypes = [P, C.c_int]
    L.or_next_id.restype = C.c_uint32
    L.or_next_id.argtypes = [P]
    L.or_read.argtypes = [P, C.c_int, P, P, P, P, P]
    L.or_nleaves.restype = C.c_int64
    L.or_nleaves.argtypes = [P]
    L.or_leaves.argtypes = [P, P, P]
    L.or_nq.restype = C.c_int64
    L.or_nq.argtypes = [P]
    L.or_deposit.argtypes = [P, P]
    L.or_field_set.argtypes = [P, C.c_int, P]
    L.or_field_table.argtypes = [P, P]
    L.or_field_solve_1d.argtypes = [P, C.c_double, P, P]
    L.or_field_solve_2d.argtypes = [P, P, C.c_double, C.c_int, P, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.or_assemble_2d.restype = C.c_int64
    L.or_assemble_2d.argtypes = [P, P, P, P, P]
    L.or_leapfrog_start.argtypes = [P]
    L.or_step.argtypes = [P, C.c_int64, C.c_int, P, C.c_int, C.POINTER(Stats)]
    L.or_adapt.argtypes = [P, C.c_int, C.c_int, C.POINTER(AdaptStats)]
    L.or_locate.argtypes = [P, C.c_int64, P, P]
    L.or_derived.argtypes = [P, C.c_int, P]
    L.or_philox4x32.argtypes = [P, P, P]
    L.or_philox4x64.argtypes = [P, P, P]
    L.or_rho.argtypes = [P, P]
    L.or_corner_phi.argtypes = [P, P]
    L.or_set_next_id.argtypes = [P, C.c_uint32]
    L.or_gather.argtypes = [P, C.c_int64, P, P]
    L.or_dipic_field.argtypes = [P, C.c_double, P, P]
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_desc(d):
    c = Desc()
    for k in ("dim", "precision", "ncells", "min_level", "max_level", "base_level", "refine_disk",
              "disk_level", "particle_bc"):
        setattr(c, k, int(d[k]))
    for k in ("length", "dt", "disk_cx", "disk_cy", "disk_r", "depth_z", "gas_density", "gas_temperature",
              "gas_mass"):
        setattr(c, k, float(d[k]))
    for i in range(4):
        c.field_bc[i] = int(d["field_bc"][i])
        c.wall_phi[i] = float(d["wall_phi"][i])
    c.disk_cz = float(d.get("disk_cz", 0.5))
    c.seed = int(d["seed"])
    c.instance_key = int(d["instance_key"])
    c.field_scheme = int(d.get("field_scheme", 0))
    c.nspecies = len(d["species"])
    for i, sp in enumerate(d["species"]):
        for k in ("charge", "mass", "w0", "sigma_el", "sigma_iz", "eps_iz", "sigma_cx", "eps_max"):
            setattr(c.species[i], k, float(sp[k]))
        c.species[i].mcc = int(sp["mcc"])
    keep = []
    if d.get("leaf_keys") is not None:
        keys = np.ascontiguousarray(d["leaf_keys"], dtype=np.uint32)
        lv = np.ascontiguousarray(d["leaf_levels"], dtype=np.uint8)
        keep = [keys, lv]
        c.leaf_keys = keys.ctypes.data
        c.leaf_levels = lv.ctypes.data
        c.nleaves = len(keys)
    c._keep = keep   # the arrays outlive the call that reads them
    return c


def philox4x32(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32(_ptr(ctr), _ptr(key), _ptr(out))
    return out


def philox4x64(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint64)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64(_ptr(ctr), _ptr(key), _ptr(out))
    return out


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


class Oracle:
    """One ES-PIC instance on the CPU, FP64 or FP32-mirror."""

    def __init__(self, desc, library=None):
        self.desc = desc
        self.L = library if library is not None else lib()
        self._d = make_desc(desc)
        self.h = self.L.or_create(C.byref(self._d))
        if not self.h:
            raise OracleError("or_create rejected the descriptor")
        self.dim = desc["dim"]
        self.nspecies = len(desc["species"])

    def __del__(self):
        if getattr(self, "h", None):
            self.L.or_destroy(self.h)
            self.h = None

    def load(self, species, s, v, w=None, ids=None):
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, self.dim)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        w = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
        ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
        _check(self.L.or_load(self.h, species, len(s), _ptr(s), _ptr(v), _ptr(w), _ptr(ids)), "or_load")

    def count(self, species):
        return self.L.or_count(self.h, species)

    @property
    def next_id(self):
        return self.L.or_next_id(self.h)

    def read(self, species):
        n = self.count(species)
        s = np.zeros((n, self.dim))
        v = np.zeros((n, 3))
        w = np.zeros(n, dtype=np.uint32)
        ids = np.zeros(n, dtype=np.uint32)
        cell = np.zeros(n, dtype=np.uint32)
        _check(self.L.or_read(self.h, species, _ptr(s), _ptr(v), _ptr(w), _ptr(ids), _ptr(cell)), "or_read")
        return dict(s=s, v=v, w=w, id=ids, cell=cell)

    def leaves(self):
        n = self.L.or_nleaves(self.h)
        keys = np.zeros(n, dtype=np.uint32)
        lv = np.zeros(n, dtype=np.uint8)
        self.L.or_leaves(self.h, _ptr(keys), _ptr(lv))
        return keys, lv

    def nq(self):
        return self.L.or_nq(self.h)

    def deposit(self):
        n = self.nq()
        q = np.zeros((2, n), dtype=np.uint64)
        _check(self.L.or_deposit(self.h, _ptr(q)), "or_deposit")
        return q

    def rho(self):
        out = np.zeros(self.nq())
        _check(self.L.or_rho(self.h, _ptr(out)), "or_rho")
        return out

    def corner_phi(self):
        out = np.zeros((self.nq(), 4))
        _check(self.L.or_corner_phi(self.h, _ptr(out)), "or_corner_phi")
        return out

    def set_next_id(self, next_id):
        _check(self.L.or_set_next_id(self.h, int(next_id)), "or_set_next_id")

    def field_set(self, kind, data):
        data = np.ascontiguousarray(data, dtype=np.float64)
        _check(self.L.or_field_set(self.h, kind, _ptr(data)), "or_field_set")

    def field_table(self):
        if self.dim == 1:
            n = self.nq()
        elif self.dim == 3:
            n = self.nq() * 24
        else:
            n = self.nq() * (2 if self.desc.get("field_scheme", 0) == FIELD_CIC_AMR else 8)
        out = np.zeros(n)
        self.L.or_field_table(self.h, _ptr(out))
        if self.dim == 1:
            return out
        if self.dim == 3:
            return out.reshape(-1, 8, 3)
        return out.reshape(-1, 2) if self.desc.get("field_scheme", 0) == FIELD_CIC_AMR else out.reshape(-1, 4, 2)

    def gather(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, self.dim)
        out = np.zeros(s.shape)
        _check(self.L.or_gather(self.h, len(s), _ptr(s), _ptr(out)), "or_gather")
        return out

    def field_solve_1d(self, phi_left):
        n = self.nq()
        phi = np.zeros(n)
        e = np.zeros(n)
        _check(self.L.or_field_solve_1d(self.h, float(phi_left), _ptr(phi), _ptr(e)), "or_field_solve_1d")
        return phi, e

    def dipic_field(self, phi_left):
        n = self.nq()
        phi = np.zeros(n)
        chi = np.zeros(n)
        _check(self.L.or_dipic_field(self.h, float(phi_left), _ptr(phi), _ptr(chi)), "or_dipic_field")
        return phi, chi

    def field_solve_2d(self, phi_init=None, rtol=1e-12, maxit=10000):
        n = self.nq()
        out = np.zeros(n)
        it = C.c_int(0)
        rr = C.c_double(0)
        pi = None if phi_init is None else np.ascontiguousarray(phi_init, dtype=np.float64)
        rc = self.L.or_field_solve_2d(self.h, _ptr(pi), float(rtol), int(maxit), _ptr(out), C.byref(it), C.byref(rr))
        return out, it.value, rr.value, rc

    def assemble_2d(self):
        nnz = self.L.or_assemble_2d(self.h, None, None, None, None)
        rows = np.zeros(nnz, dtype=np.int32)
        cols = np.zeros(nnz, dtype=np.int32)
        vals = np.zeros(nnz)
        rhs = np.zeros(self.nq())
        self.L.or_assemble_2d(self.h, _ptr(rows), _ptr(cols), _ptr(vals), _ptr(rhs))
        return rows, cols, vals, rhs

    def leapfrog_start(self):
        _check(self.L.or_leapfrog_start(self.h), "or_leapfrog_start")

    def step(self, step0, nsteps=1, v_next=None, solve_1d=False):
        st = Stats()
        vn = None if v_next is None else np.ascontiguousarray(v_next, dtype=np.float64)
        _check(self.L.or_step(self.h, int(step0), int(nsteps), _ptr(vn), int(bool(solve_1d)), C.byref(st)), "or_step")
        return st.as_dict()

    def adapt(self, n_lo=16, n_hi=64):
        st = AdaptStats()
        _check(self.L.or_adapt(self.h, int(n_lo), int(n_hi), C.byref(st)), "or_adapt")
        return st.as_dict()

    def locate(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, self.dim)
        out = np.zeros(len(s), dtype=np.uint32)
        _check(self.L.or_locate(self.h, len(s), _ptr(s), _ptr(out)), "or_locate")
        return out

    def derived(self, species):
        out = np.zeros(12)
        self.L.or_derived(self.h, species, _ptr(out))
        names = ["qm_dt", "dt_L", "Tcand", "a_el", "a_iz", "v_iz2", "mu2", "vmax2", "v_thg", "a_cx", "gmax",
                 "hqm_dt"]
        return dict(zip(names, out))


# field kinds
NODE_E_1D, NODE_PHI_1D, CORNER_PHI_2D, CORNER_E_2D, CELL_PHI_2D, CELL_E_1D, CELL_E_2D = 0, 1, 2, 3, 4, 5, 6
CORNER_PHI_3D, CORNER_E_3D = 7, 8
FIELD_CIC_EM, FIELD_CIC_EC, FIELD_CIC_AMR, FIELD_DIPIC = 0, 1, 2, 3
