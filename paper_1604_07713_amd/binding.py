"""Thin ctypes binding of libpic.so (the C ABI in include/pic.h).

Argument marshalling only: every step of the particle loop and of the field
solves runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing or fails to load, LibraryMissing is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")
_LIB = None

PIC_OK, PIC_E_ARG, PIC_E_NOMEM, PIC_E_CAPACITY, PIC_E_HIP, PIC_E_STATE, PIC_E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
FIELD_CIC_EM, FIELD_CIC_EC, FIELD_CIC_AMR, FIELD_DIPIC = 0, 1, 2, 3   # particle-field couplings (include/pic.h)
ABI_VERSION = 4                     # PIC_ABI_VERSION of include/pic.h
NODE_E_1D, NODE_PHI_1D, CORNER_PHI_2D, CORNER_E_2D, CELL_PHI_2D, CELL_E_1D, CELL_E_2D = 0, 1, 2, 3, 4, 5, 6
CORNER_PHI_3D, CORNER_E_3D = 7, 8


class LibraryMissing(RuntimeError):
    pass


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"status {code}: {msg}")
        self.code = code


class SpeciesDesc(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("w0", C.c_double), ("mcc", C.c_int),
                ("sigma_el", C.c_double), ("sigma_iz", C.c_double), ("eps_iz", C.c_double),
                ("sigma_cx", C.c_double), ("eps_max", C.c_double)]


class InstanceDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("precision", C.c_int), ("length", C.c_double), ("dt", C.c_double),
                ("ncells", C.c_int), ("min_level", C.c_int), ("max_level", C.c_int), ("base_level", C.c_int),
                ("refine_disk", C.c_int), ("disk_cx", C.c_double), ("disk_cy", C.c_double),
                ("disk_r", C.c_double), ("disk_level", C.c_int), ("field_bc", C.c_int * 4),
                ("wall_phi", C.c_double * 4), ("particle_bc", C.c_int), ("depth_z", C.c_double),
                ("gas_density", C.c_double), ("gas_temperature", C.c_double), ("gas_mass", C.c_double),
                ("seed", C.c_uint64), ("instance_key", C.c_uint32), ("nspecies", C.c_int),
                ("species", SpeciesDesc * 2), ("capacity", C.c_int64 * 2), ("field_scheme", C.c_int),
                ("leaf_keys", C.c_void_p), ("leaf_levels", C.c_void_p), ("nleaves", C.c_int64),
                ("disk_cz", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("alive_start", C.c_int64 * 2), ("absorbed", C.c_int64 * 2), ("elastic", C.c_int64),
                ("ionization", C.c_int64), ("cx", C.c_int64), ("births", C.c_int64),
                ("numax_violations", C.c_int64 * 2), ("lost_reflect", C.c_int64), ("loop_ms", C.c_double),
                ("step_ms", C.c_double), ("loop_launches", C.c_int64), ("room_stops", C.c_int64)]

    def as_dict(self):
        return dict(alive_start=list(self.alive_start), absorbed=list(self.absorbed), elastic=self.elastic,
                    ionization=self.ionization, cx=self.cx, births=self.births,
                    numax_violations=list(self.numax_violations), lost_reflect=self.lost_reflect,
                    loop_ms=self.loop_ms, step_ms=self.step_ms, loop_launches=self.loop_launches,
                    room_stops=self.room_stops)


class StepArgs(C.Structure):
    _fields_ = [("step0", C.c_int64), ("nsteps", C.c_int), ("solve_field", C.c_int),
                ("v_next", C.c_void_p), ("sort_every", C.c_int), ("batched", C.c_int), ("grid", C.c_int),
                ("graph_steps", C.c_int), ("slots", C.c_void_p), ("nslots", C.c_int), ("timing", C.c_int)]


class AdaptArgs(C.Structure):
    _fields_ = [("n_lo", C.c_int), ("n_hi", C.c_int)]


class AdaptStats(C.Structure):
    _fields_ = [("refined", C.c_int64), ("coarsened", C.c_int64), ("balance_refined", C.c_int64),
                ("split_parents", C.c_int64), ("merged_pairs", C.c_int64), ("nleaves", C.c_int64),
                ("merge_energy_change", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = {
    # name: (restype, argtypes)
    "pic_abi_version": (C.c_int, []),
    "pic_last_error": (C.c_char_p, [C.c_void_p]),
    "pic_mesh_build": (C.c_int, [C.POINTER(InstanceDesc), C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pic_destroy": (None, [C.c_void_p]),
    "pic_particles_load": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "pic_field_set": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "pic_leapfrog_start": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_step": (C.c_int, [C.c_void_p, C.POINTER(StepArgs), C.POINTER(StepStats)]),
    "pic_step_noalloc": (C.c_int, [C.c_void_p, C.POINTER(StepArgs), C.POINTER(StepStats)]),
    "pic_deposit": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "pic_step_index": (C.c_int64, [C.c_void_p, C.c_int]),
    "pic_set_slot_limit": (C.c_int, [C.c_void_p, C.c_int, C.c_int64]),
    "pic_deposit_read": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "pic_set_births_ranking": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "pic_field_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_double, C.c_int, C.c_void_p,
                                  C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "pic_adapt": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(AdaptArgs), C.POINTER(AdaptStats)]),
    "pic_count": (C.c_int64, [C.c_void_p, C.c_int, C.c_int]),
    "pic_next_id": (C.c_uint32, [C.c_void_p, C.c_int]),
    "pic_particles_read": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "pic_nleaves": (C.c_int64, [C.c_void_p, C.c_int]),
    "pic_leaves_read": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "pic_nq": (C.c_int64, [C.c_void_p, C.c_int]),
    "pic_field_read": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "pic_sort": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_locate": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p]),
    "pic_gather": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p]),
    "pic_derived": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "pic_philox": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pic_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pic_sync": (C.c_int, [C.c_void_p]),
    "pic_num_slots": (C.c_int, [C.c_void_p]),
    "pic_admit": (C.c_int, [C.c_void_p, C.POINTER(InstanceDesc), C.POINTER(C.c_int)]),
    "pic_retire": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_slot_bytes": (C.c_int64, [C.c_void_p, C.c_int]),
    "pic_set_allocator": (C.c_int, [C.c_void_p, C.c_void_p]),
}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Device memory of a context from torch's caching allocator, in stream
    order on the context's stream (pic_set_allocator)."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else device

        def _alloc(nbytes, stream, user):
            try:
                return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
            except Exception:
                return None

        def _free(p, user):
            self._torch.cuda.caching_allocator_delete(p)
        self._alloc = ALLOC_FN(_alloc)   # kept alive with this object
        self._free = FREE_FN(_free)
        self.struct = Allocator(self._alloc, self._free, None)


def lib():
    """Load libpic.so (raises LibraryMissing if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        try:
            L = C.CDLL(LIB_PATH)
        except OSError as e:
            raise LibraryMissing(f"cannot load {LIB_PATH}: {e}") from e
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.pic_abi_version() != ABI_VERSION:   # the structures below must match the library's
            raise LibraryMissing(f"{LIB_PATH} has ABI {L.pic_abi_version()}, this binding {ABI_VERSION}; rebuild")
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_desc(d, capacity=(0, 0)):
    c = InstanceDesc()
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
    c.nspecies = len(d["species"])
    for i, sp in enumerate(d["species"]):
        for k in ("charge", "mass", "w0", "sigma_el", "sigma_iz", "eps_iz", "sigma_cx", "eps_max"):
            setattr(c.species[i], k, float(sp[k]))
        c.species[i].mcc = int(sp["mcc"])
    cap = d.get("capacity", capacity)
    c.capacity[0] = int(cap[0])
    c.capacity[1] = int(cap[1])
    c.field_scheme = int(d.get("field_scheme", FIELD_CIC_EM))
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


def default_stream():
    """Handle of torch's current HIP stream on the current device, or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Context:
    """A library context owning one or more instance slots on the GPU."""

    def __init__(self, descs, stream=None, allocator=None):
        """allocator: None (hipMalloc and the library's block cache), or e.g.
        TorchAllocator() (device memory from torch's caching allocator)."""
        if isinstance(descs, dict):
            descs = [descs]
        self.descs = list(descs)
        self._allocator = allocator
        first = [] if allocator is not None else self.descs
        made = [make_desc(d) for d in first]
        arr = (InstanceDesc * max(len(first), 1))(*made)
        h = C.c_void_p()
        L = lib()
        rc = L.pic_mesh_build(arr, len(first), stream if stream is not None else default_stream(), C.byref(h))
        if rc != PIC_OK:
            raise PicError(rc, L.pic_last_error(None).decode())
        self.h = h
        self._slot_desc = {i: d for i, d in enumerate(first)}
        if allocator is not None:
            self._check(L.pic_set_allocator(self.h, C.byref(allocator.struct)))
            for d in self.descs:
                self.admit(d)

    def close(self):
        if getattr(self, "h", None):
            lib().pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != PIC_OK:
            raise PicError(rc, lib().pic_last_error(self.h).decode())
        return rc

    def desc(self, slot):
        return self._slot_desc[slot]

    def dim(self, slot):
        return self._slot_desc[slot]["dim"]

    # ---- the five calls of the method ----
    def load(self, slot, species, s, v, w=None, ids=None):
        dim = self.dim(slot)
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, dim)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        w = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
        ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
        self._check(lib().pic_particles_load(self.h, slot, species, len(s), _p(s), _p(v), _p(w), _p(ids)))

    def step(self, step0, nsteps=1, v_next=None, solve_field=False, sort_every=0, batched=0, slots=None,
             timing=False, grid=0, graph_steps=0, noalloc=False):
        """pic_step, or pic_step_noalloc with noalloc=True."""
        a = StepArgs()
        a.step0 = int(step0)
        a.nsteps = int(nsteps)
        a.solve_field = int(bool(solve_field))
        vn = None
        if v_next is not None:
            vn = np.ascontiguousarray(v_next, dtype=np.float64)
            a.v_next = vn.ctypes.data
        a.sort_every = int(sort_every)
        a.batched = int(batched)
        a.grid = int(grid)
        a.graph_steps = int(graph_steps)
        sl = None
        if slots is not None:
            sl = np.ascontiguousarray(slots, dtype=np.int32)
            a.slots = sl.ctypes.data
            a.nslots = len(sl)
        a.timing = int(timing)   # True = 1: every launch; n: every n-th step
        st = StepStats()
        fn = lib().pic_step_noalloc if noalloc else lib().pic_step
        self._check(fn(self.h, C.byref(a), C.byref(st)))
        return st.as_dict()

    def deposit(self, slot=0, rho=False):
        """Integer charge sums [2][nq]; with rho=True also the charge density [nq]."""
        n = self.nq(slot)
        q = np.zeros((2, n), dtype=np.uint64)
        r = np.zeros(n) if rho else None
        self._check(lib().pic_deposit(self.h, slot, _p(q), _p(r)))
        return (q, r) if rho else q

    def set_births_ranking(self, slot, method):
        """0: by the births of recent steps, 1: pairwise, 2: binned."""
        self._check(lib().pic_set_births_ranking(self.h, slot, int(method)))

    def deposit_read(self, slot=0):
        n = self.nq(slot)
        q = np.zeros((2, n), dtype=np.uint64)
        self._check(lib().pic_deposit_read(self.h, slot, _p(q)))
        return q

    def adapt(self, slot=0, n_lo=16, n_hi=64):
        a = AdaptArgs(int(n_lo), int(n_hi))
        st = AdaptStats()
        self._check(lib().pic_adapt(self.h, slot, C.byref(a), C.byref(st)))
        return st.as_dict()

    # ---- helpers ----
    def field_set(self, slot, kind, data):
        data = np.ascontiguousarray(data, dtype=np.float64)
        self._check(lib().pic_field_set(self.h, slot, kind, _p(data)))

    def field_table(self, slot=0):
        cic = self.dim(slot) == 2 and self._slot_desc[slot].get("field_scheme", 0) == FIELD_CIC_AMR
        n = (self.nq(slot) if self.dim(slot) == 1 else self.nq(slot) * 24 if self.dim(slot) == 3
             else self.nq(slot) * (2 if cic else 8))
        out = np.zeros(n)
        self._check(lib().pic_field_read(self.h, slot, _p(out)))
        if self.dim(slot) == 1:
            return out
        if self.dim(slot) == 3:
            return out.reshape(-1, 8, 3)
        return out.reshape(-1, 2) if cic else out.reshape(-1, 4, 2)

    def gather(self, slot, s):
        dim = self.dim(slot)
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, dim)
        out = np.zeros(s.shape)
        self._check(lib().pic_gather(self.h, slot, len(s), _p(s), _p(out)))
        return out

    def field_solve_1d(self, slot, phi_left):
        n = self.nq(slot)
        phi = np.zeros(n)
        e = np.zeros(n)
        it, rr = C.c_int(0), C.c_double(0)
        self._check(lib().pic_field_solve(self.h, slot, float(phi_left), None, 0.0, 0, _p(phi), _p(e),
                                          C.byref(it), C.byref(rr)))
        return phi, e

    def field_solve_2d(self, slot=0, phi_init=None, rtol=1e-12, maxit=10000, want_e=False):
        n = self.nq(slot)
        phi = np.zeros(n)
        e = np.zeros(n * 8) if want_e else None
        it, rr = C.c_int(0), C.c_double(0)
        pi = None if phi_init is None else np.ascontiguousarray(phi_init, dtype=np.float64)
        rc = lib().pic_field_solve(self.h, slot, 0.0, _p(pi), float(rtol), int(maxit), _p(phi), _p(e),
                                   C.byref(it), C.byref(rr))
        if rc not in (PIC_OK, PIC_E_NUMERIC):
            self._check(rc)
        return phi, it.value, rr.value, rc

    def leapfrog_start(self, slot=0):
        self._check(lib().pic_leapfrog_start(self.h, slot))

    def count(self, slot, species):
        n = lib().pic_count(self.h, slot, species)
        if n < 0:
            self._check(int(n))
        return n

    def next_id(self, slot=0):
        return lib().pic_next_id(self.h, slot)

    def step_index(self, slot=0):
        n = lib().pic_step_index(self.h, slot)
        if n < 0:
            self._check(int(n))
        return int(n)

    def set_slot_limit(self, slot, max_bytes):
        self._check(lib().pic_set_slot_limit(self.h, slot, int(max_bytes)))

    def read(self, slot, species):
        dim = self.dim(slot)
        n = self.count(slot, species)
        s = np.zeros((n, dim))
        v = np.zeros((n, 3))
        w = np.zeros(n, dtype=np.uint32)
        ids = np.zeros(n, dtype=np.uint32)
        cell = np.zeros(n, dtype=np.uint32)
        self._check(lib().pic_particles_read(self.h, slot, species, _p(s), _p(v), _p(w), _p(ids), _p(cell)))
        return dict(s=s, v=v, w=w, id=ids, cell=cell)

    def nq(self, slot=0):
        return int(lib().pic_nq(self.h, slot))

    def leaves(self, slot=0):
        n = int(lib().pic_nleaves(self.h, slot))
        keys = np.zeros(n, dtype=np.uint32)
        lv = np.zeros(n, dtype=np.uint8)
        self._check(lib().pic_leaves_read(self.h, slot, _p(keys), _p(lv)))
        return keys, lv

    def sort(self, slot=0):
        self._check(lib().pic_sort(self.h, slot))

    def locate(self, slot, s):
        s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1, self.dim(slot))
        out = np.zeros(len(s), dtype=np.uint32)
        self._check(lib().pic_locate(self.h, slot, len(s), _p(s), _p(out)))
        return out

    def derived(self, slot, species):
        out = np.zeros(12)
        self._check(lib().pic_derived(self.h, slot, species, _p(out)))
        names = ["qm_dt", "dt_L", "Tcand", "a_el", "a_iz", "v_iz2", "mu2", "vmax2", "v_thg", "a_cx", "gmax",
                 "hqm_dt"]
        return dict(zip(names, out))

    def sync(self):
        self._check(lib().pic_sync(self.h))

    def admit(self, desc):
        s = C.c_int(-1)
        md = make_desc(desc)
        self._check(lib().pic_admit(self.h, C.byref(md), C.byref(s)))
        self._slot_desc[s.value] = desc
        return s.value

    def retire(self, slot):
        self._check(lib().pic_retire(self.h, slot))
        self._slot_desc.pop(slot, None)

    def slot_bytes(self, slot):
        return int(lib().pic_slot_bytes(self.h, slot))


def philox4x32(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(ctr)
    rc = lib().pic_philox(len(ctr), _p(ctr), _p(key), _p(out))
    if rc != PIC_OK:
        raise PicError(rc, lib().pic_last_error(None).decode())
    return out
