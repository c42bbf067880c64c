"""FP64 CPU oracle for the shallow-water step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it, and the two share no code: the oracle is
plain C (``swe_oracle.c``, compiled with ``gcc -ffp-contract=off``) driven
through ctypes from here.

Parity pins for each function are in ``tests/test_oracle_*.py``.  The inflow
conditions impose their discharge as the edge mass flux, so the volume they
deliver is pinned exactly (the hydrograph's, sum over steps of Q(t^n) dt) in
sub- and supercritical flow alike.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction): the
    serial library, and the same source with OpenMP (its edge and cell loops
    on all cores, every sum still taken in the serial order, so both give
    bitwise the same results)."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out):
            tmp = out + ".tmp"
            cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC"] + extra + \
                  ["-shared", "-o", tmp, _SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(tmp, out)
    return _LIB


_libs = {}


def lib(omp: bool = False):
    """The serial oracle library, or its OpenMP build (omp=True)."""
    L = _libs.get(omp)
    if L is None:
        path = _LIB_OMP if omp else _LIB
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        L.om_mesh_new.restype = ctypes.c_void_p
        L.om_mesh_new.argtypes = [_c_double_p, ctypes.c_int64, _c_int32_p, ctypes.c_int64,
                                  _c_int32_p, _c_int32_p, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int]
        L.om_mesh_free.argtypes = [ctypes.c_void_p]
        L.om_mesh_n_edges.restype = ctypes.c_int64
        L.om_mesh_n_edges.argtypes = [ctypes.c_void_p]
        L.om_mesh_n_boundary_edges.restype = ctypes.c_int64
        L.om_mesh_n_boundary_edges.argtypes = [ctypes.c_void_p]
        L.om_mesh_geometry.argtypes = [ctypes.c_void_p] + [_c_double_p] * 6 + [_c_int32_p]
        L.om_sim_new.restype = ctypes.c_void_p
        L.om_sim_new.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                 _c_double_p, ctypes.c_int32, _c_int32_p, _c_int32_p, _c_double_p,
                                 _c_int32_p, _c_double_p, _c_double_p, _c_double_p, ctypes.c_double,
                                 ctypes.c_char_p, ctypes.c_int]
        L.om_sim_free.argtypes = [ctypes.c_void_p]
        L.om_next_dt.restype = ctypes.c_double
        L.om_next_dt.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.om_step.restype = ctypes.c_int
        L.om_step.argtypes = [ctypes.c_void_p, ctypes.c_double, _c_double_p]
        L.om_run_until.restype = ctypes.c_int
        L.om_run_until.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, _c_int64_p]
        L.om_get_state.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p]
        L.om_set_state.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p, ctypes.c_double]
        L.om_diag.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p, _c_int64_p]
        L.om_hllc.argtypes = [ctypes.c_double] * 7 + [_c_double_p]
        L.om_friction.restype = ctypes.c_double
        L.om_friction.argtypes = [ctypes.c_double] * 5
        L.om_friction_cf.restype = ctypes.c_double
        L.om_friction_cf.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.om_friction_closure.restype = ctypes.c_double
        L.om_friction_closure.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 5
        L.om_sim_set_scalars.restype = ctypes.c_int
        L.om_sim_set_scalars.argtypes = [ctypes.c_void_p, ctypes.c_int32, _c_double_p, _c_double_p,
                                         ctypes.c_char_p, ctypes.c_int]
        L.om_get_scalars.argtypes = [ctypes.c_void_p, _c_double_p]
        L.om_scalar_diag.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]
        L.om_sim_set_sources.restype = ctypes.c_int
        L.om_sim_set_sources.argtypes = [ctypes.c_void_p, _c_int32_p, ctypes.c_int32, _c_int32_p, _c_int32_p,
                                         _c_int32_p, _c_double_p, _c_double_p, ctypes.c_char_p, ctypes.c_int]
        L.om_source_volume.restype = ctypes.c_double
        L.om_source_volume.argtypes = [ctypes.c_void_p]
        L.om_sim_set_morpho.restype = ctypes.c_int
        L.om_sim_set_morpho.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_double] * 6 + \
            [_c_double_p, ctypes.c_char_p, ctypes.c_int]
        L.om_get_bed.argtypes = [ctypes.c_void_p, _c_double_p]
        L.om_sim_set_drain.restype = ctypes.c_int
        L.om_sim_set_drain.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        L.om_morpho_diag.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]
        L.om_sed_cell.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 12 + [_c_double_p] * 4
        L.om_sim_set_friction.restype = ctypes.c_int
        L.om_sim_set_friction.argtypes = [ctypes.c_void_p, ctypes.c_int32, _c_double_p, ctypes.c_char_p, ctypes.c_int]
        L.om_sim_set_bed.restype = ctypes.c_int
        L.om_sim_set_bed.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, ctypes.c_char_p, ctypes.c_int]
        L.om_sim_set_diffusion.restype = ctypes.c_int
        L.om_sim_set_diffusion.argtypes = [ctypes.c_void_p, _c_double_p, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, _c_double_p, ctypes.c_char_p, ctypes.c_int]
        L.om_get_psi.argtypes = [ctypes.c_void_p, _c_double_p]
        L.om_bc_flux.restype = ctypes.c_double
        L.om_bc_flux.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.om_threads.restype = ctypes.c_int
        L.om_threads.argtypes = [ctypes.c_int]
        _libs[omp] = L
    return L


def threads(n: int = 0) -> int:
    """Threads of the OpenMP oracle (n > 0 sets them)."""
    return lib(True).om_threads(n)


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_c_double_p)


def _ip(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_c_int32_p)


class OracleError(RuntimeError):
    pass


def hllc(hL, unL, utL, hR, unR, utR, g=9.81):
    F = np.zeros(3)
    lib().om_hllc(hL, unL, utL, hR, unR, utR, g, _dp(F))
    return F


def friction_factor(qabs, h, gn2, dt, h_min=1e-4):
    return lib().om_friction(qabs, h, gn2, dt, h_min)


# friction closures of Table friction_closure, by name
FRICTION = {"manning": 0, "strickler": 1, "chezy": 2, "bezzola": 3}
SED = {"mpm": 0, "grass": 1, "eh": 2}


def sed_cell(closure, alpha, m, thr, d_m, s_rel, g, h, u, v, cf2, nx, ny):
    """(q_B.n, dq_B,n/dq_n, lambda_1, lambda_2) of one cell."""
    out = [ctypes.c_double() for _ in range(4)]
    lib().om_sed_cell(SED[closure], alpha, m, thr, d_m, s_rel, g, h, u, v, cf2, nx, ny,
                      *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def friction_cf(kind, par, h):
    """c_f of a log-type closure ("chezy": par = K_s, "bezzola": par = y_R)."""
    return lib().om_friction_cf(FRICTION[kind], par, h)


def friction_closure(kind, coef, qabs, h, dt, h_min=1e-4):
    """Split factor of one closure; coef is g n^2 / g k^-2 for the power
    laws and K_s / y_R for the log types, as the step stores it."""
    return lib().om_friction_closure(FRICTION[kind], coef, qabs, h, dt, h_min)


class Mesh:
    """Oracle mesh; omp=True uses the OpenMP build (its states too)."""

    def __init__(self, nodes, tri, bnd_seg=None, bnd_tag=None, omp: bool = False):
        L = self._L = lib(omp)
        self.nodes = np.ascontiguousarray(nodes, np.float64)
        self.tri = np.ascontiguousarray(tri, np.int32)
        seg = np.zeros((0, 2), np.int32) if bnd_seg is None else np.ascontiguousarray(bnd_seg, np.int32)
        tag = np.zeros((0,), np.int32) if bnd_tag is None else np.ascontiguousarray(bnd_tag, np.int32)
        err = ctypes.create_string_buffer(256)
        self._p = L.om_mesh_new(_dp(self.nodes), len(self.nodes), _ip(self.tri), len(self.tri),
                                _ip(seg), _ip(tag), len(seg), err, 256)
        if not self._p:
            raise OracleError(err.value.decode())
        self.n_cells = len(self.tri)

    @property
    def n_edges(self):
        return self._L.om_mesh_n_edges(self._p)

    @property
    def n_boundary_edges(self):
        return self._L.om_mesh_n_boundary_edges(self._p)

    def geometry(self):
        n = self.n_cells
        out = dict(area=np.zeros(n), zb=np.zeros(n), rho=np.zeros((n, 3)), nx=np.zeros((n, 3)),
                   ny=np.zeros((n, 3)), length=np.zeros((n, 3)), nbr=np.zeros((n, 3), np.int32))
        self._L.om_mesh_geometry(self._p, _dp(out["area"]), _dp(out["zb"]), _dp(out["rho"]), _dp(out["nx"]),
                               _dp(out["ny"]), _dp(out["length"]), _ip(out["nbr"]))
        return out

    def __del__(self):
        if getattr(self, "_p", None):
            self._L.om_mesh_free(self._p)
            self._p = None


class Sim:
    """One FP64 oracle run of a scenario (see swe_inputs.Scenario)."""

    def __init__(self, sc, t0: float = 0.0, mesh: Optional[Mesh] = None, dt_max: Optional[float] = None,
                 omp: bool = False):
        self.mesh = mesh or Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, omp=omp)
        L = self._L = self.mesh._L
        n = sc.n_cells
        bcs = sc.bcs
        tags = np.array([b.tag for b in bcs], np.int32)
        kinds = np.array([b.kind for b in bcs], np.int32)
        slopes = np.array([b.slope for b in bcs], np.float64)
        npts = np.array([0 if b.t is None else len(b.t) for b in bcs], np.int32)
        bt = np.concatenate([np.asarray(b.t, np.float64) for b in bcs if b.t is not None] or [np.zeros(0)])
        bQ = np.concatenate([np.asarray(b.Q, np.float64) for b in bcs if b.Q is not None] or [np.zeros(0)])
        H0 = None if sc.H0 is None else np.ascontiguousarray(sc.H0, np.float64)
        h0 = None if sc.h0 is None else np.ascontiguousarray(sc.h0, np.float64)
        pars = np.array([getattr(b, "par", 0.0) for b in bcs], np.float64)
        self._keep = [tags, kinds, slopes, npts, bt, bQ, H0, h0, pars]
        self._bcs = list(bcs)
        qx0 = np.ascontiguousarray(sc.qx0, np.float64)
        qy0 = np.ascontiguousarray(sc.qy0, np.float64)
        man = np.ascontiguousarray(sc.manning, np.float64)
        err = ctypes.create_string_buffer(256)
        self._p = L.om_sim_new(self.mesh._p, sc.g, sc.cfl, sc.h_min, sc.dt_max if dt_max is None else dt_max,
                               _dp(H0), _dp(h0), _dp(qx0), _dp(qy0), _dp(man), len(bcs),
                               _ip(tags), _ip(kinds), _dp(slopes), _ip(npts), _dp(bt), _dp(bQ), _dp(pars),
                               t0, err, 256)
        if not self._p:
            raise OracleError(err.value.decode())
        self.n = n
        kind = getattr(sc, "friction", "manning")
        if kind != "manning":
            if L.om_sim_set_friction(self._p, FRICTION[kind], _dp(man), err, 256):
                raise OracleError(err.value.decode())
        self.ns = 0
        phi0 = getattr(sc, "phi0", None)
        if phi0 is not None:
            phi0 = np.ascontiguousarray(np.atleast_2d(phi0), np.float64)
            ns = phi0.shape[0]
            pin = np.zeros((max(len(bcs), 1), ns))
            for b, bc in enumerate(bcs):
                if len(getattr(bc, "phi_in", ())):
                    pin[b] = bc.phi_in
            pin = np.ascontiguousarray(pin)
            self._keep += [phi0, pin]
            if L.om_sim_set_scalars(self._p, ns, _dp(phi0), _dp(pin), err, 256):
                raise OracleError(err.value.decode())
            self.ns = ns
        if getattr(sc, "diffusion", None) is not None:
            self.set_diffusion(sc.diffusion)
        if len(getattr(sc, "sources", ())):
            self.set_sources(sc.src_region, sc.sources)
        if getattr(sc, "morpho", None) is not None:
            self.set_morpho(sc.morpho)
        if getattr(sc, "drain", False):
            self.set_drain(True)

    def set_diffusion(self, df, psi0=None):
        """Diffusion of the species (swe_inputs.Diffusion: per-species
        molecular diffusivity Km, dispersion alpha_L, alpha_T, relaxation
        time zeta); psi0 (species, cells, 2) initial auxiliary variables."""
        km = np.ascontiguousarray(np.broadcast_to(np.asarray(df.Km, np.float64), (self.ns,)))
        p0 = None if psi0 is None else np.ascontiguousarray(psi0, np.float64)
        self._keep += [km, p0]
        err = ctypes.create_string_buffer(256)
        if self._L.om_sim_set_diffusion(self._p, _dp(km), df.alpha_L, df.alpha_T, df.zeta, _dp(p0), err, 256):
            raise OracleError(err.value.decode())

    def psi(self):
        """Auxiliary variables (psi_x, psi_y) of the diffusing species,
        (species, cells, 2)."""
        p = np.zeros((self.ns, self.n, 2))
        self._L.om_get_psi(self._p, _dp(p))
        return p

    def set_drain(self, on):
        """Draining-time positivity limiter on or off."""
        err = ctypes.create_string_buffer(256)
        if self._L.om_sim_set_drain(self._p, int(bool(on)), err, 256):
            raise OracleError(err.value.decode())

    def set_morpho(self, mo):
        """Exner module with the closure and parameters of mo (swe_inputs.Morpho)."""
        zr = None if mo.z_rel is None else np.ascontiguousarray(mo.z_rel, np.float64)
        self._keep.append(zr)
        err = ctypes.create_string_buffer(256)
        if self._L.om_sim_set_morpho(self._p, SED[mo.closure], mo.alpha, mo.m, mo.thr, mo.d_m, mo.s_rel,
                                   mo.porosity, _dp(zr), err, 256):
            raise OracleError(err.value.decode())

    def set_bed(self, z, H=None):
        """Cell beds per cell instead of the node means, with surfaces H (or
        None to keep each cell's depth)."""
        z = np.ascontiguousarray(z, np.float64)
        H = None if H is None else np.ascontiguousarray(H, np.float64)
        err = ctypes.create_string_buffer(256)
        if self._L.om_sim_set_bed(self._p, _dp(z), _dp(H), err, 256):
            raise OracleError(err.value.decode())

    def bed(self):
        z = np.zeros(self.n)
        self._L.om_get_bed(self._p, _dp(z))
        return z

    def morpho_diag(self):
        """Sediment volume (1 - p) sum z |cell|, the volume that left through
        open boundaries, and the volume the fixed-bed clip added."""
        v, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._L.om_morpho_diag(self._p, ctypes.byref(v), ctypes.byref(b), ctypes.byref(c))
        return v.value, b.value, c.value

    def set_sources(self, region, sources):
        """External water sources and sinks: region (cells,) -> index into
        sources (-1: none); each source has mode, unit, t, v."""
        region = np.ascontiguousarray(region, np.int32)
        mode = np.array([x.mode for x in sources], np.int32)
        unit = np.array([x.unit for x in sources], np.int32)
        npts = np.array([0 if x.t is None else len(x.t) for x in sources], np.int32)
        t = np.concatenate([np.asarray(x.t, np.float64) for x in sources if x.t is not None] or [np.zeros(0)])
        v = np.concatenate([np.asarray(x.v, np.float64) for x in sources if x.v is not None] or [np.zeros(0)])
        self._keep += [region, mode, unit, npts, t, v]
        err = ctypes.create_string_buffer(256)
        if self._L.om_sim_set_sources(self._p, _ip(region), len(sources), _ip(mode), _ip(unit), _ip(npts), _dp(t),
                                    _dp(v), err, 256):
            raise OracleError(err.value.decode())

    def source_volume(self):
        """Volume the external sources added so far (negative: removed)."""
        return self._L.om_source_volume(self._p)

    def __del__(self):
        if getattr(self, "_p", None):
            self._L.om_sim_free(self._p)
            self._p = None

    def next_dt(self, t_end=float("inf")):
        return self._L.om_next_dt(self._p, t_end)

    def step(self, t_end=float("inf")):
        dt = ctypes.c_double()
        rc = self._L.om_step(self._p, t_end, ctypes.byref(dt))
        if rc:
            e = OracleError(f"oracle step failed ({rc})")
            e.code = rc
            raise e
        return dt.value

    def run_until(self, t_end, max_steps=0):
        n = ctypes.c_int64()
        rc = self._L.om_run_until(self._p, t_end, max_steps, ctypes.byref(n))
        if rc:
            e = OracleError(f"oracle run failed ({rc})")
            e.code = rc
            raise e
        return n.value

    def run_steps(self, k, t_end=float("inf")):
        return self.run_until(t_end, max_steps=k)

    def state(self):
        H, qx, qy = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        t = ctypes.c_double()
        self._L.om_get_state(self._p, _dp(H), _dp(qx), _dp(qy), ctypes.byref(t))
        return H, qx, qy, t.value

    def set_state(self, H, qx, qy, t):
        H, qx, qy = (np.ascontiguousarray(a, np.float64) for a in (H, qx, qy))
        self._L.om_set_state(self._p, _dp(H), _dp(qx), _dp(qy), t)

    @property
    def t(self):
        return self.state()[3]

    def scalars(self):
        """Specific masses q = h phi, (species, cells)."""
        q = np.zeros((self.ns, self.n))
        self._L.om_get_scalars(self._p, _dp(q))
        return q

    def scalar_diag(self):
        """Per species: total mass, the mass that left through open boundaries,
        and the mass set by resetting cells left dry."""
        m, b, c = (np.zeros(max(self.ns, 1)) for _ in range(3))
        self._L.om_scalar_diag(self._p, _dp(m), _dp(b), _dp(c))
        return m[:self.ns], b[:self.ns], c[:self.ns]

    def bc_flux(self, tag):
        """Boundary-flux integral over the edges tagged `tag` (the first
        condition given for the tag), positive where water left."""
        for b, bc in enumerate(self._bcs):
            if bc.tag == tag:
                return self._L.om_bc_flux(self._p, b)
        return 0.0

    def diag(self):
        m, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        s = ctypes.c_int64()
        self._L.om_diag(self._p, ctypes.byref(m), ctypes.byref(b), ctypes.byref(c), ctypes.byref(s))
        return dict(mass=m.value, bnd_flux=b.value, clipped=c.value, steps=s.value)
