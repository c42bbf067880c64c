"""Thin ctypes binding of the gfx950 shallow-water library (``include/swe.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libswe.so``.  Device memory comes from PyTorch's caching allocator and
work is issued on PyTorch's current HIP stream, through the library's
allocation callbacks.  There is no CPU fallback: importing this module on a
tree without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswe.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ENEGDEPTH, EBUDGET, ENODT, ESINK = 0, -1, -2, -3, -4, -5, -6, -7, -8
BC_WALL, BC_INFLOW_UNIFORM, BC_OUTFLOW_ZEROGRAD, BC_ZHYDROGRAPH = 0, 1, 2, 3
BC_INFLOW_FROUDE, BC_OUTFLOW_UNIFORM, BC_OUTFLOW_WEIR, BC_OUTFLOW_HQ, BC_DYNAMIC_WALL = 4, 5, 6, 7, 8
FP64, FP32 = 0, 1
NEG_CLIP, NEG_ERROR = 0, 1
LIMIT_NONE, LIMIT_DRAIN = 0, 1
FRICTION = {"manning": 0, "strickler": 1, "chezy": 2, "bezzola": 3}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SweDevice(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p), ("hip_stream", ctypes.c_void_p)]


class SweBC(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int32), ("kind", ctypes.c_int32), ("slope", ctypes.c_double),
                ("t", _dp), ("Q", _dp), ("n_pts", ctypes.c_int32), ("par", ctypes.c_double)]


class SweSource(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("unit", ctypes.c_int32), ("t", _dp), ("v", _dp),
                ("n_pts", ctypes.c_int32)]


class SweMorpho(ctypes.Structure):
    _fields_ = [("closure", ctypes.c_int32), ("alpha", ctypes.c_double), ("m", ctypes.c_double),
                ("thr", ctypes.c_double), ("d_m", ctypes.c_double), ("s_rel", ctypes.c_double),
                ("porosity", ctypes.c_double)]


SED = {"mpm": 0, "grass": 1, "eh": 2}


class SweParams(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("cfl", ctypes.c_double), ("h_min", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("precision", ctypes.c_int32), ("neg_depth_policy", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("steps_per_graph", ctypes.c_int32), ("renumber", ctypes.c_int32), ("friction", ctypes.c_int32),
                ("limiter", ctypes.c_int32)]


# every symbol the header declares, with (restype, argtypes)
SIGNATURES = {
    "swe_params_default": (None, [ctypes.POINTER(SweParams)]),
    "swe_mesh_create": (ctypes.c_int32, [_dp, ctypes.c_int64, _ip, ctypes.c_int64, _ip, _ip, ctypes.c_int64,
                                         ctypes.POINTER(SweParams), ctypes.POINTER(SweDevice),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "swe_mesh_destroy": (None, [ctypes.c_void_p]),
    "swe_mesh_info": (None, [ctypes.c_void_p, _lp, _lp, _lp]),
    "swe_state_footprint": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32]),
    "swe_mesh_check": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "swe_state_init": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(SweParams), _dp, _dp, _dp, _dp, _dp,
                                        ctypes.POINTER(SweBC), ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "swe_state_destroy": (None, [ctypes.c_void_p]),
    "swe_step": (ctypes.c_int32, [ctypes.c_void_p, _dp]),
    "swe_run_until": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, _lp]),
    "swe_launch_steps": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64]),
    "swe_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "swe_prepare_graphs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "swe_state_read": (ctypes.c_int32, [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]),
    "swe_mass": (ctypes.c_int32, [ctypes.c_void_p, _dp, _dp, _dp, _lp]),
    "swe_boundary_flux": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "swe_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _ip]),
    "swe_state_set_scalars": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _dp, _dp]),
    "swe_state_read_scalars": (ctypes.c_int32, [ctypes.c_void_p, _dp]),
    "swe_state_set_diffusion": (ctypes.c_int32, [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, _dp]),
    "swe_state_read_psi": (ctypes.c_int32, [ctypes.c_void_p, _dp]),
    "swe_scalar_mass": (ctypes.c_int32, [ctypes.c_void_p, _dp, _dp, _dp]),
    "swe_state_set_sources": (ctypes.c_int32, [ctypes.c_void_p, _ip, ctypes.POINTER(SweSource), ctypes.c_int32]),
    "swe_source_volume": (ctypes.c_int32, [ctypes.c_void_p, _dp]),
    "swe_state_set_morpho": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(SweMorpho), _dp]),
    "swe_state_read_bed": (ctypes.c_int32, [ctypes.c_void_p, _dp]),
    "swe_morpho_volume": (ctypes.c_int32, [ctypes.c_void_p, _dp, _dp, _dp]),
    "swe_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(SweDevice),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "swe_batch_destroy": (None, [ctypes.c_void_p]),
    "swe_batch_add": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, _ip]),
    "swe_batch_remove": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "swe_batch_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _ip]),
    "swe_batch_launch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "swe_batch_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _ip]),
    "swe_batch_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, _ip, _ip, _dp, _lp]),
    "swe_batch_footprint": (ctypes.c_int64, [ctypes.c_void_p]),
    "swe_batch_step_noalloc": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), _dp, ctypes.c_int32, ctypes.c_int32,
                                                _ip]),
    "swe_last_error": (ctypes.c_char_p, []),
    "swe_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Loads libswe.so (no build, no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(python paper_2102_12862_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SweError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"swe error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise SweError(rc, load().swe_last_error().decode())


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _i(a):
    return None if a is None else a.ctypes.data_as(_ip)


class TorchDevice:
    """Bridges the library's allocation callbacks to PyTorch's caching
    allocator and hands it the current HIP stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to PyTorch")
        self._torch = torch
        self._live = {}
        self.stream = stream if stream is not None else torch.cuda.current_stream()

        def _alloc(nbytes, ctx):
            try:
                t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device="cuda")
            except RuntimeError:
                return None
            p = t.data_ptr()
            self._live[p] = t
            return p

        def _free(ptr, ctx):
            self._live.pop(ptr, None)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = SweDevice(self._alloc, self._free, None, ctypes.c_void_p(self.stream.cuda_stream))

    @property
    def live_bytes(self):
        return sum(t.numel() for t in self._live.values())


def params(**kw) -> SweParams:
    p = SweParams()
    load().swe_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Mesh:
    def __init__(self, nodes, tri, bnd_seg=None, bnd_tag=None, device: Optional[TorchDevice] = None,
                 renumber: bool = True):
        L = load()
        # device=False: host-side mesh preparation only (no device callbacks);
        # states created on such a mesh use hipMalloc and the default stream
        self.device = None if device is False else (device or TorchDevice())
        nodes = np.ascontiguousarray(nodes, np.float64)
        tri = np.ascontiguousarray(tri, np.int32)
        seg = np.zeros((0, 2), np.int32) if bnd_seg is None else np.ascontiguousarray(bnd_seg, np.int32)
        tag = np.zeros((0,), np.int32) if bnd_tag is None else np.ascontiguousarray(bnd_tag, np.int32)
        p = params(renumber=1 if renumber else 0)
        h = ctypes.c_void_p()
        _check(L.swe_mesh_create(_d(nodes), len(nodes), _i(tri), len(tri), _i(seg), _i(tag), len(seg),
                                 ctypes.byref(p), None if self.device is None else ctypes.byref(self.device.struct),
                                 ctypes.byref(h)))
        self._h = h
        self._destroy = load().swe_mesh_destroy
        self.n_cells = len(tri)

    def info(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        load().swe_mesh_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return dict(n_cells=a.value, n_edges=b.value, n_boundary_edges=c.value)

    def footprint(self, precision=FP32):
        return load().swe_state_footprint(self._h, precision)

    def check(self, tile=256):
        _check(load().swe_mesh_check(self._h, tile))

    def close(self):
        if getattr(self, "_h", None):
            # the bound destroy call outlives the module's globals at interpreter exit
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def _bc_array(bcs):
    arr = (SweBC * max(1, len(bcs)))()
    keep = []
    for k, b in enumerate(bcs):
        t = None if b.t is None else np.ascontiguousarray(b.t, np.float64)
        Q = None if b.Q is None else np.ascontiguousarray(b.Q, np.float64)
        keep += [t, Q]
        arr[k] = SweBC(b.tag, b.kind, b.slope, _d(t), _d(Q), 0 if t is None else len(t), getattr(b, "par", 0.0))
    return arr, keep


class State:
    """Device-resident solve of one scenario (see swe_inputs.Scenario)."""

    def __init__(self, mesh: Mesh, sc, precision=FP64, t0: float = 0.0, H0=None, h0=None, qx0=None, qy0=None,
                 **pkw):
        L = load()
        self.mesh = mesh
        self.precision = precision
        pkw.setdefault("friction", FRICTION[getattr(sc, "friction", "manning")])
        pkw.setdefault("limiter", LIMIT_DRAIN if getattr(sc, "drain", False) else LIMIT_NONE)
        p = params(g=sc.g, cfl=sc.cfl, h_min=sc.h_min, dt_max=sc.dt_max, precision=precision, **pkw)
        if H0 is None and h0 is None:
            H0, h0 = sc.H0, sc.h0
        qx0 = sc.qx0 if qx0 is None else qx0
        qy0 = sc.qy0 if qy0 is None else qy0
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (H0, h0, qx0, qy0, sc.manning)]
        bc, keep = _bc_array(sc.bcs)
        h = ctypes.c_void_p()
        _check(L.swe_state_init(mesh._h, ctypes.byref(p), *[_d(a) for a in arrs], bc, len(sc.bcs), t0,
                                ctypes.byref(h)))
        self._h = h
        self._destroy = load().swe_state_destroy
        self.n = mesh.n_cells
        self.ns = 0
        phi0 = getattr(sc, "phi0", None)
        if phi0 is not None:
            pin = np.zeros((len(sc.bcs), np.atleast_2d(phi0).shape[0]))
            for b, bc in enumerate(sc.bcs):
                if len(getattr(bc, "phi_in", ())):
                    pin[b] = bc.phi_in
            self.set_scalars(phi0, pin)
            if getattr(sc, "diffusion", None) is not None:
                self.set_diffusion(sc.diffusion)
        if len(getattr(sc, "sources", ())):
            self.set_sources(sc.src_region, sc.sources)
        if getattr(sc, "morpho", None) is not None:
            self.set_morpho(sc.morpho)

    def set_morpho(self, mo):
        """Exner module with mo (closure, alpha, m, thr, d_m, s_rel, porosity,
        z_rel), or off for None."""
        if mo is None:
            _check(load().swe_state_set_morpho(self._h, None, None))
            return
        p = SweMorpho(SED[mo.closure], mo.alpha, mo.m, mo.thr, mo.d_m, mo.s_rel, mo.porosity)
        zr = None if mo.z_rel is None else np.ascontiguousarray(mo.z_rel, np.float64)
        _check(load().swe_state_set_morpho(self._h, ctypes.byref(p), _d(zr)))

    def bed(self):
        z = np.empty(self.n)
        _check(load().swe_state_read_bed(self._h, _d(z)))
        return z

    def morpho_volume(self):
        """Sediment volume, the volume that left through open boundaries, and
        the volume the fixed-bed clip added."""
        v, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load().swe_morpho_volume(self._h, ctypes.byref(v), ctypes.byref(b), ctypes.byref(c)))
        return v.value, b.value, c.value

    def set_sources(self, region, sources):
        """External water sources and sinks: region (cells,) indexes sources
        (-1: none); each source has mode, unit, t, v."""
        region = np.ascontiguousarray(region, np.int32)
        arr = (SweSource * max(1, len(sources)))()
        keep = [region]
        for k, x in enumerate(sources):
            t = None if x.t is None else np.ascontiguousarray(x.t, np.float64)
            v = None if x.v is None else np.ascontiguousarray(x.v, np.float64)
            keep += [t, v]
            arr[k] = SweSource(x.mode, x.unit, _d(t), _d(v), 0 if t is None else len(t))
        _check(load().swe_state_set_sources(self._h, _i(region), arr, len(sources)))

    def source_volume(self):
        """Volume the sources added since they were set (negative: removed)."""
        v = ctypes.c_double()
        _check(load().swe_source_volume(self._h, ctypes.byref(v)))
        return v.value

    def set_scalars(self, phi0, phi_in=None):
        """Passive species with initial concentrations phi0 (species, cells)
        and inflow concentrations phi_in (boundary conditions, species)."""
        phi0 = np.ascontiguousarray(np.atleast_2d(phi0), np.float64)
        ns = phi0.shape[0] if phi0.size else 0
        pin = None if phi_in is None else np.ascontiguousarray(phi_in, np.float64)
        _check(load().swe_state_set_scalars(self._h, ns, _d(phi0), _d(pin)))
        self.ns = ns

    def set_diffusion(self, df, psi0=None):
        """Diffusion of the species (df: Km per species or one value,
        alpha_L, alpha_T, zeta); psi0 (species, cells, 2) the initial
        auxiliary variables."""
        km = np.ascontiguousarray(np.broadcast_to(np.asarray(df.Km, np.float64), (self.ns,)))
        p0 = None if psi0 is None else np.ascontiguousarray(psi0, np.float64)
        _check(load().swe_state_set_diffusion(self._h, _d(km), df.alpha_L, df.alpha_T, df.zeta, _d(p0)))

    def psi(self):
        """Auxiliary variables of the diffusing species, (species, cells, 2)."""
        p = np.zeros((self.ns, self.n, 2))
        _check(load().swe_state_read_psi(self._h, _d(p)))
        return p

    def scalars(self):
        """Specific masses q = h phi, (species, cells)."""
        q = np.zeros((self.ns, self.n))
        _check(load().swe_state_read_scalars(self._h, _d(q)))
        return q

    def scalar_mass(self):
        """Per species: total mass, the mass that left through open
        boundaries, and the mass set by resetting cells left dry."""
        m, b, c = (np.zeros(max(self.ns, 1)) for _ in range(3))
        _check(load().swe_scalar_mass(self._h, _d(m), _d(b), _d(c)))
        return m[:self.ns], b[:self.ns], c[:self.ns]

    def step(self):
        dt = ctypes.c_double()
        _check(load().swe_step(self._h, ctypes.byref(dt)))
        return dt.value

    def run_until(self, t_end):
        n = ctypes.c_int64()
        _check(load().swe_run_until(self._h, t_end, ctypes.byref(n)))
        return n.value

    def launch_steps(self, k, t_end=float("inf")):
        _check(load().swe_launch_steps(self._h, t_end, k))

    def sync(self):
        _check(load().swe_sync(self._h))

    def read(self):
        H, h, qx, qy = (np.empty(self.n) for _ in range(4))
        t = ctypes.c_double()
        _check(load().swe_state_read(self._h, _d(H), _d(h), _d(qx), _d(qy), ctypes.byref(t)))
        return dict(H=H, h=h, qx=qx, qy=qy, t=t.value)

    def mass(self):
        m, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        s = ctypes.c_int64()
        _check(load().swe_mass(self._h, ctypes.byref(m), ctypes.byref(b), ctypes.byref(c), ctypes.byref(s)))
        return dict(mass=m.value, bnd_flux=b.value, clipped=c.value, steps=s.value)

    def boundary_flux(self, tag):
        """Boundary-flux integral over the edges tagged `tag` (positive:
        water left the domain)."""
        v = ctypes.c_double()
        _check(load().swe_boundary_flux(self._h, tag, ctypes.byref(v)))
        return v.value

    def autotune(self, k=8):
        b = ctypes.c_int32()
        _check(load().swe_autotune(self._h, k, ctypes.byref(b)))
        return b.value

    def prepare_graphs(self, steps_per_graph=0):
        _check(load().swe_prepare_graphs(self._h, steps_per_graph))

    def close(self):
        if getattr(self, "_h", None):
            # the bound destroy call outlives the module's globals at interpreter exit
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Many independent states stepped together by one persistent kernel per
    step, each with its own time step."""

    def __init__(self, precision=FP32, budget_bytes: int = 0, device: Optional[TorchDevice] = None):
        self.device = device or TorchDevice()
        h = ctypes.c_void_p()
        _check(load().swe_batch_create(precision, budget_bytes, ctypes.byref(self.device.struct), ctypes.byref(h)))
        self._h = h
        self._destroy = load().swe_batch_destroy
        self.members = {}

    def add(self, state: State, t_end: float) -> int:
        slot = ctypes.c_int32()
        _check(load().swe_batch_add(self._h, state._h, t_end, ctypes.byref(slot)))
        self.members[slot.value] = state
        return slot.value

    def remove(self, slot: int):
        _check(load().swe_batch_remove(self._h, slot))
        self.members.pop(slot, None)

    def step(self, k: int) -> int:
        n = ctypes.c_int32()
        _check(load().swe_batch_step(self._h, k, ctypes.byref(n)))
        return n.value

    def launch(self, k: int):
        _check(load().swe_batch_launch(self._h, k))

    def autotune(self, k=4):
        b = ctypes.c_int32()
        _check(load().swe_batch_autotune(self._h, k, ctypes.byref(b)))
        return b.value

    def poll(self, slot: int):
        d, e = ctypes.c_int32(), ctypes.c_int32()
        t, s = ctypes.c_double(), ctypes.c_int64()
        _check(load().swe_batch_poll(self._h, slot, ctypes.byref(d), ctypes.byref(e), ctypes.byref(t), ctypes.byref(s)))
        return dict(done=bool(d.value), error=e.value, t=t.value, steps=s.value)

    def footprint(self):
        return load().swe_batch_footprint(self._h)

    def close(self):
        if getattr(self, "_h", None):
            # the bound destroy call outlives the module's globals at interpreter exit
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def batch_step_noalloc(states, t_end, k: int) -> int:
    """k persistent batched steps of `states` (each until its t_end) with
    the work list in the library's fixed device scratch: no device memory is
    allocated.  Returns how many states are still running."""
    n = len(states)
    hs = (ctypes.c_void_p * max(n, 1))(*[st._h.value for st in states])
    te = np.ascontiguousarray(np.broadcast_to(np.asarray(t_end, np.float64), (n,)))
    act = ctypes.c_int32()
    _check(load().swe_batch_step_noalloc(hs, _d(te), n, k, ctypes.byref(act)))
    return act.value


def exported_symbols(path: str = LIB_PATH) -> Sequence[str]:
    """Names of the C-ABI functions the library exports (read with ctypes)."""
    L = ctypes.CDLL(path)
    return [n for n in SIGNATURES if hasattr(L, n)]
