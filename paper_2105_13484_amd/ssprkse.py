"""ctypes binding of ``libssprkse.so`` (the C ABI declared in include/ssprkse.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies device memory (one tensor per mesh and per
state) and the stream.  ``torch`` is imported before the library is loaded
so that the process holds a single HIP runtime.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_size_t, c_uint8, c_void_p, c_char_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSE_LIB_PATH") or os.path.join(_HERE, "libssprkse.so")

SSE_OK, SSE_EINVAL, SSE_ENOMEM, SSE_EDEVICE, SSE_ENONFINITE, SSE_ESTATE = range(6)
SSE_FP64, SSE_MIXED, SSE_MIXED_BT64 = 0, 1, 2
SSE_ZSTAR, SSE_ISOPYCNAL = 0, 1
SSE_RECONCILE_OFF, SSE_RECONCILE_EXACT, SSE_RECONCILE_LITERAL = 0, 1, 2
SSE_VMIX_EXPLICIT, SSE_VMIX_IMPLICIT = 0, 1
SSE_HDIFF_DEL2, SSE_HDIFF_DEL4 = 0, 1
SSE_TRACER_NONE, SSE_TRACER_TEMPERATURE = 0, 1
PROF_CLASSES = ("fe_edge", "fe_cell", "fe_vertex", "bt_eval", "thickness", "other")

EXPORTED = (
    "sse_last_error", "sse_version", "sse_mesh_validate", "sse_mesh_device_bytes", "sse_mesh_create",
    "sse_mesh_destroy", "sse_state_workspace_bytes", "sse_state_create", "sse_state_destroy", "sse_state_init",
    "sse_step", "sse_step_async", "sse_sync", "sse_read_state", "sse_profile_enable", "sse_profile_read",
    "sse_debug_baroclinic_feuler", "sse_debug_barotropic_substep", "sse_debug_thickness_stage",
    "sse_state_set_edge_variant", "sse_state_get_edge_variant", "sse_state_set_geometry", "sse_state_use_graph",
    "sse_batch_create", "sse_batch_destroy", "sse_batch_add", "sse_batch_remove", "sse_batch_size",
    "sse_batch_set_geometry", "sse_batch_program_bytes", "sse_batch_compile", "sse_batch_launches_per_step",
    "sse_batch_use_graph", "sse_batch_step_async", "sse_batch_sync", "sse_batch_step", "sse_footprint_bytes",
    "sse_state_set_bt_variant", "sse_state_get_bt_variant", "sse_state_set_tracer", "sse_read_tracer",
    "sse_barotropic_substep_noalloc", "sse_debug_set_barrier_spins", "sse_debug_edge_gathers",
)

# Edge-pass variants: -1 direct gathers, 0 / 1 / 2 LDS tiles of 8 / 16 / 32 edges.
EDGE_VARIANTS = (-1, 0, 1, 2)


class SSEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ssprkse error {code}: {msg}")
        self.code = code


class sse_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("n_cells", c_int32), ("n_edges", c_int32), ("n_vertices", c_int32),
        ("max_edges", c_int32), ("max_edges2", c_int32),
        ("cells_on_edge", POINTER(c_int32)), ("edges_on_cell", POINTER(c_int32)),
        ("n_edges_on_cell", POINTER(c_int32)), ("vertices_on_edge", POINTER(c_int32)),
        ("edges_on_vertex", POINTER(c_int32)), ("edges_on_edge", POINTER(c_int32)),
        ("n_edges_on_edge", POINTER(c_int32)), ("weights_on_edge", POINTER(c_double)),
        ("dc_edge", POINTER(c_double)), ("dv_edge", POINTER(c_double)), ("f_edge", POINTER(c_double)),
        ("area_cell", POINTER(c_double)), ("bottom_depth", POINTER(c_double)),
        ("area_triangle", POINTER(c_double)), ("cell_mask", POINTER(c_uint8)),
    ]


class sse_params(ctypes.Structure):
    _fields_ = [
        ("n_layers", c_int32), ("scheme", c_int32), ("substeps", c_int32), ("precision", c_int32),
        ("vcoord", c_int32), ("reconcile", c_int32), ("vmix", c_int32), ("hdiff", c_int32),
        ("tracer", c_int32),
        ("dt", c_double), ("gravity", c_double), ("rho0", c_double), ("nu_h", c_double),
        ("nu_v", c_double), ("c_drag", c_double),
        ("kappa_h", c_double), ("kappa_v", c_double), ("eos_alpha", c_double), ("eos_tref", c_double),
    ]


_lib = None


def load():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (one HIP runtime per process: torch's)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    dp = POINTER(c_double)
    sig = {
        "sse_last_error": (c_char_p, []),
        "sse_version": (c_char_p, []),
        "sse_mesh_validate": (c_int, [POINTER(sse_mesh_desc)]),
        "sse_mesh_device_bytes": (c_int, [POINTER(sse_mesh_desc), POINTER(c_size_t)]),
        "sse_mesh_create": (c_int, [POINTER(sse_mesh_desc), P, c_size_t, P, POINTER(P)]),
        "sse_mesh_destroy": (c_int, [P]),
        "sse_state_workspace_bytes": (c_int, [P, POINTER(sse_params), POINTER(c_size_t)]),
        "sse_state_create": (c_int, [P, POINTER(sse_params), P, c_size_t, P, POINTER(P)]),
        "sse_state_destroy": (c_int, [P]),
        "sse_state_init": (c_int, [P, dp, dp, dp, dp]),
        "sse_step": (c_int, [P, c_int32]),
        "sse_step_async": (c_int, [P, c_int32]),
        "sse_sync": (c_int, [P]),
        "sse_read_state": (c_int, [P, dp, dp, dp, dp]),
        "sse_profile_enable": (c_int, [P, c_int]),
        "sse_profile_read": (c_int, [P, POINTER(c_int32), dp]),
        "sse_debug_baroclinic_feuler": (c_int, [P, dp, dp, dp, dp, c_double, dp, dp]),
        "sse_debug_barotropic_substep": (c_int, [P, c_int32, c_int32, c_double, dp, dp, dp, dp, dp, dp]),
        "sse_debug_thickness_stage": (c_int, [P, dp, dp, dp, c_double, dp, dp]),
        "sse_barotropic_substep_noalloc": (c_int, [P, c_int32, c_int32, c_double, P, P, P, P, P, P]),
        "sse_debug_set_barrier_spins": (c_int, [P, ctypes.c_uint32]),
        "sse_debug_edge_gathers": (c_int, [P]),
        "sse_state_set_edge_variant": (c_int, [P, c_int]),
        "sse_state_get_edge_variant": (c_int, [P, POINTER(c_int)]),
        "sse_state_set_bt_variant": (c_int, [P, c_int]),
        "sse_state_set_tracer": (c_int, [P, POINTER(c_double)]),
        "sse_read_tracer": (c_int, [P, POINTER(c_double)]),
        "sse_state_get_bt_variant": (c_int, [P, POINTER(c_int)]),
        "sse_state_set_geometry": (c_int, [P, c_int, c_int]),
        "sse_state_use_graph": (c_int, [P, c_int]),
        "sse_batch_create": (c_int, [P, POINTER(P)]),
        "sse_batch_destroy": (c_int, [P]),
        "sse_batch_add": (c_int, [P, P]),
        "sse_batch_remove": (c_int, [P, P]),
        "sse_batch_size": (c_int, [P, POINTER(c_int32)]),
        "sse_batch_set_geometry": (c_int, [P, c_int, c_int]),
        "sse_batch_program_bytes": (c_int, [P, POINTER(c_size_t)]),
        "sse_batch_compile": (c_int, [P, P, c_size_t]),
        "sse_batch_launches_per_step": (c_int, [P, POINTER(c_int32)]),
        "sse_batch_use_graph": (c_int, [P, c_int]),
        "sse_batch_step_async": (c_int, [P, c_int32]),
        "sse_batch_sync": (c_int, [P]),
        "sse_batch_step": (c_int, [P, c_int32]),
        "sse_footprint_bytes": (c_int, [POINTER(sse_mesh_desc), POINTER(sse_params), POINTER(c_size_t)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().sse_last_error().decode()


def _check(rc: int, allow=()):
    if rc != SSE_OK and rc not in allow:
        raise SSEError(rc, last_error())
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def mesh_desc(mesh, bottom_depth, cell_mask):
    """Build an ``sse_mesh_desc`` from a synthetic mesh; returns (desc, keepalive)."""
    keep = {
        "coe": np.ascontiguousarray(mesh.cellsOnEdge, np.int32),
        "eoc": np.ascontiguousarray(mesh.edgesOnCell, np.int32),
        "neoc": np.ascontiguousarray(mesh.nEdgesOnCell, np.int32),
        "voe": np.ascontiguousarray(mesh.verticesOnEdge, np.int32),
        "eov": np.ascontiguousarray(mesh.edgesOnVertex, np.int32),
        "eoe": np.ascontiguousarray(mesh.edgesOnEdge, np.int32),
        "neoe": np.ascontiguousarray(mesh.nEdgesOnEdge, np.int32),
        "w": _f64(mesh.weightsOnEdge), "dc": _f64(mesh.dcEdge), "dv": _f64(mesh.dvEdge),
        "f": _f64(mesh.fEdge), "ac": _f64(mesh.areaCell), "H": _f64(bottom_depth),
        "at": _f64(mesh.areaTriangle), "mask": np.ascontiguousarray(cell_mask, np.uint8),
    }
    d = sse_mesh_desc()
    d.n_cells, d.n_edges, d.n_vertices = mesh.nCells, mesh.nEdges, mesh.nVertices
    d.max_edges, d.max_edges2 = keep["eoc"].shape[1], keep["eoe"].shape[1]
    d.cells_on_edge, d.edges_on_cell, d.n_edges_on_cell = _iptr(keep["coe"]), _iptr(keep["eoc"]), _iptr(keep["neoc"])
    d.vertices_on_edge, d.edges_on_vertex = _iptr(keep["voe"]), _iptr(keep["eov"])
    d.edges_on_edge, d.n_edges_on_edge = _iptr(keep["eoe"]), _iptr(keep["neoe"])
    d.weights_on_edge, d.dc_edge, d.dv_edge, d.f_edge = _dptr(keep["w"]), _dptr(keep["dc"]), _dptr(keep["dv"]), _dptr(keep["f"])
    d.area_cell, d.bottom_depth, d.area_triangle = _dptr(keep["ac"]), _dptr(keep["H"]), _dptr(keep["at"])
    d.cell_mask = keep["mask"].ctypes.data_as(POINTER(c_uint8))
    return d, keep


def make_params(p) -> sse_params:
    out = sse_params()
    for name, _ in sse_params._fields_:
        setattr(out, name, getattr(p, name))
    return out


def footprint_bytes(mesh, params) -> int:
    """Device bytes (mesh image + workspace) of one state of `params` on `mesh`
    (sized from the mesh topology; depths and the land mask do not matter)."""
    d, keep = mesh_desc(mesh, np.ones(mesh.nCells), np.ones(mesh.nCells, np.uint8))
    p = make_params(params)
    n = c_size_t()
    _check(load().sse_footprint_bytes(byref(d), byref(p), byref(n)))
    del keep
    return int(n.value)


def sse_mesh_validate(mesh, bottom_depth, cell_mask) -> int:
    d, _keep = mesh_desc(mesh, bottom_depth, cell_mask)
    return load().sse_mesh_validate(byref(d))


def _aligned_buffer(nbytes: int, device):
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


class DeviceMesh:
    """A mesh uploaded into a caller-owned (torch) device buffer."""

    def __init__(self, mesh, bottom_depth, cell_mask, device="cuda", stream=None):
        lib = load()
        d, keep = mesh_desc(mesh, bottom_depth, cell_mask)
        nbytes = c_size_t()
        _check(lib.sse_mesh_device_bytes(byref(d), byref(nbytes)))
        self.buf, ptr = _aligned_buffer(nbytes.value, device)
        self.handle = c_void_p()
        _check(lib.sse_mesh_create(byref(d), c_void_p(ptr), nbytes.value, _stream_ptr(stream), byref(self.handle)))
        self.nbytes = nbytes.value
        self.C, self.E, self.V = mesh.nCells, mesh.nEdges, mesh.nVertices
        self._keep = keep

    def close(self):
        if self.handle:
            load().sse_mesh_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceState:
    """One model state (prognostic fields + stage buffers) on a DeviceMesh."""

    def __init__(self, dmesh: DeviceMesh, params, device="cuda", stream=None):
        lib = load()
        self.mesh = dmesh
        self.params = params
        self.p = make_params(params)
        self.L = params.n_layers
        nbytes = c_size_t()
        _check(lib.sse_state_workspace_bytes(dmesh.handle, byref(self.p), byref(nbytes)))
        self.buf, ptr = _aligned_buffer(nbytes.value, device)
        self.handle = c_void_p()
        self.stream = stream
        _check(lib.sse_state_create(dmesh.handle, byref(self.p), c_void_p(ptr), nbytes.value, _stream_ptr(stream),
                                    byref(self.handle)))
        self.nbytes = nbytes.value

    def init(self, h, u, rho, h_ref=None):
        h, u, rho = _f64(h), _f64(u), _f64(rho)
        hr = _f64(h_ref) if h_ref is not None else None
        _check(load().sse_state_init(self.handle, _dptr(h), _dptr(u), _dptr(rho),
                                     _dptr(hr) if hr is not None else None))

    def set_tracer(self, T):
        """Tracer runs: the layer temperature [C][L] (sets the density by the EOS)."""
        T = _f64(T)
        _check(load().sse_state_set_tracer(self.handle, _dptr(T)))

    def read_tracer(self):
        T = np.empty((self.mesh.C, self.L))
        _check(load().sse_read_tracer(self.handle, _dptr(T)))
        return T

    def step(self, n: int = 1) -> int:
        """Advance n steps; returns SSE_OK or SSE_ENONFINITE."""
        return _check(load().sse_step(self.handle, int(n)), allow=(SSE_ENONFINITE,))

    def step_async(self, n: int = 1):
        _check(load().sse_step_async(self.handle, int(n)))

    def sync(self) -> int:
        return _check(load().sse_sync(self.handle), allow=(SSE_ENONFINITE,))

    def read(self):
        C, E, L = self.mesh.C, self.mesh.E, self.L
        h, u = np.empty((C, L)), np.empty((E, L))
        zeta, ubar = np.empty(C), np.empty(E)
        _check(load().sse_read_state(self.handle, _dptr(h), _dptr(u), _dptr(zeta), _dptr(ubar)))
        return {"h": h, "u": u, "zeta": zeta, "ubar": ubar}

    def profile(self, classes=PROF_CLASSES):
        """Time every launch of the named kernel classes (empty = off)."""
        mask = 0
        for c in classes:
            mask |= 1 << PROF_CLASSES.index(c)
        _check(load().sse_profile_enable(self.handle, mask))

    @property
    def edge_variant(self) -> int:
        v = c_int(0)
        _check(load().sse_state_get_edge_variant(self.handle, ctypes.byref(v)))
        return int(v.value)

    @edge_variant.setter
    def edge_variant(self, variant: int):
        _check(load().sse_state_set_edge_variant(self.handle, int(variant)))

    def set_geometry(self, cols_per_block: int = 4, block_2d: int = 256):
        """Launch geometry (wavefronts per column-kernel workgroup, threads per 2D workgroup)."""
        _check(load().sse_state_set_geometry(self.handle, int(cols_per_block), int(block_2d)))

    def use_graph(self, enable: bool = True):
        """Replay each step as one captured HIP graph (needs a non-default stream)."""
        _check(load().sse_state_use_graph(self.handle, int(bool(enable))))

    @property
    def bt_variant(self) -> int:
        """Barotropic loop kernels: 0 one launch per evaluation, 1 one per substep."""
        v = c_int(0)
        _check(load().sse_state_get_bt_variant(self.handle, ctypes.byref(v)))
        return int(v.value)

    @bt_variant.setter
    def bt_variant(self, variant: int):
        _check(load().sse_state_set_bt_variant(self.handle, int(variant)))

    def debug_edge_gathers(self):
        """Enqueue one gather-only edge pass on the state's stream (a
        measurement aid: the direct edge pass's column loads without its
        arithmetic; the state is left as it was)."""
        _check(load().sse_debug_edge_gathers(self.handle))

    def set_barrier_spins(self, spins: int = 0):
        """Polls before a grid barrier of the persistent barotropic loop gives up (0: default)."""
        _check(load().sse_debug_set_barrier_spins(self.handle, int(spins)))

    def try_bt_variant(self, variant: int) -> bool:
        """Select a barotropic loop variant; False (and no change) if unavailable."""
        return load().sse_state_set_bt_variant(self.handle, int(variant)) == 0

    def try_edge_variant(self, variant: int) -> bool:
        """Select an edge-pass variant; False (and no change) if it does not fit."""
        rc = load().sse_state_set_edge_variant(self.handle, int(variant))
        return rc == 0

    def profile_read(self):
        n = (c_int32 * len(PROF_CLASSES))()
        ms = (c_double * len(PROF_CLASSES))()
        _check(load().sse_profile_read(self.handle, n, ms))
        return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(PROF_CLASSES)}

    # -- per-kernel debug entry points ---------------------------------------
    def debug_baroclinic_feuler(self, u, ubar, zeta, h, dt):
        E, L = self.mesh.E, self.L
        u, ubar, zeta, h = _f64(u), _f64(ubar), _f64(zeta), _f64(h)
        ut1, G = np.empty((E, L)), np.empty(E)
        _check(load().sse_debug_baroclinic_feuler(self.handle, _dptr(u), _dptr(ubar), _dptr(zeta), _dptr(h),
                                                  float(dt), _dptr(ut1), _dptr(G)))
        return ut1, G

    def debug_barotropic_substep(self, scheme, M, dt, ubar, zeta, G):
        C, E = self.mesh.C, self.mesh.E
        ubar, zeta, G = _f64(ubar), _f64(zeta), _f64(G)
        u1, z1, F = np.empty(E), np.empty(C), np.empty(E)
        _check(load().sse_debug_barotropic_substep(self.handle, int(scheme), int(M), float(dt), _dptr(ubar),
                                                   _dptr(zeta), _dptr(G), _dptr(u1), _dptr(z1), _dptr(F)))
        return u1, z1, F

    def barotropic_substep_noalloc(self, scheme, M, dt, ubar, zeta, G, ubar1, zeta1, Fzeta):
        """The allocation-free barotropic loop on device tensors (float64,
        contiguous, on the state's device; caller numbering).  Enqueued on the
        state's stream; returns without waiting."""
        import torch
        C, E = self.mesh.C, self.mesh.E
        for t, n in ((ubar, E), (zeta, C), (G, E), (ubar1, E), (zeta1, C), (Fzeta, E)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
                raise ValueError("expected contiguous float64 device tensors of the mesh's sizes")
        _check(load().sse_barotropic_substep_noalloc(self.handle, int(scheme), int(M), float(dt), ubar.data_ptr(),
                                                     zeta.data_ptr(), G.data_ptr(), ubar1.data_ptr(),
                                                     zeta1.data_ptr(), Fzeta.data_ptr()))

    def debug_thickness_stage(self, h_in, u, uA, dt):
        C, L = self.mesh.C, self.L
        h_in, u, uA = _f64(h_in), _f64(u), _f64(uA)
        h_out, z = np.empty((C, L)), np.empty(C)
        _check(load().sse_debug_thickness_stage(self.handle, _dptr(h_in), _dptr(u), _dptr(uA), float(dt),
                                                _dptr(h_out), _dptr(z)))
        return h_out, z

    def close(self):
        if self.handle:
            load().sse_state_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def state_from_case(case, device="cuda", stream=None, params=None):
    """Upload a synthetic case: returns (DeviceMesh, DeviceState) with the initial state set."""
    dm = DeviceMesh(case.mesh, case.H, case.cell_mask, device=device, stream=stream)
    st = DeviceState(dm, params if params is not None else case.params, device=device, stream=stream)
    st.init(case.h, case.u, case.rho, case.h_ref)
    if getattr(st.params, "tracer", 0):
        st.set_tracer(case.temp)
    return dm, st


class Batch:
    """Several DeviceStates advanced together, one launch per step phase.

    Members must share precision, scheme and vertical coordinate and must have
    been created on the batch's stream.  ``compile()`` allocates the device
    buffer for the merged launch program (a torch tensor) and uploads it.

    Members may be added while steps enqueued by ``step_async`` run: the
    program those launches read stays allocated until the next ``sync`` (or
    ``step``), and the new program is compiled at the next launch.
    """

    def __init__(self, stream=None):
        self.stream = stream
        self.handle = c_void_p()
        _check(load().sse_batch_create(_stream_ptr(stream), byref(self.handle)))
        self.members = []
        self.buf = None
        self._retired = []     # programs that launches in flight may still read

    def _retire(self):
        if self.buf is not None:
            self._retired.append(self.buf)
        self.buf = None

    def add(self, state: "DeviceState"):
        _check(load().sse_batch_add(self.handle, state.handle))
        self.members.append(state)
        self._retire()

    def remove(self, state: "DeviceState"):
        _check(load().sse_batch_remove(self.handle, state.handle))
        self.members = [m for m in self.members if m is not state]
        self._retire()

    def __len__(self):
        return len(self.members)

    def set_geometry(self, cols_per_block: int = 4, block_2d: int = 256):
        _check(load().sse_batch_set_geometry(self.handle, int(cols_per_block), int(block_2d)))
        self._retire()

    def compile(self, device="cuda"):
        lib = load()
        nbytes = c_size_t()
        _check(lib.sse_batch_program_bytes(self.handle, byref(nbytes)))
        self._retire()
        self.buf, ptr = _aligned_buffer(max(nbytes.value, 256), device)
        _check(lib.sse_batch_compile(self.handle, c_void_p(ptr), nbytes.value))
        return nbytes.value

    def launches_per_step(self) -> int:
        n = c_int32()
        _check(load().sse_batch_launches_per_step(self.handle, byref(n)))
        return int(n.value)

    def use_graph(self, enable: bool = True):
        _check(load().sse_batch_use_graph(self.handle, int(bool(enable))))

    def step(self, n: int = 1) -> int:
        if self.buf is None:
            self.compile()
        rc = _check(load().sse_batch_step(self.handle, int(n)), allow=(SSE_ENONFINITE,))
        self._retired.clear()
        return rc

    def step_async(self, n: int = 1):
        if self.buf is None:
            self.compile()
        _check(load().sse_batch_step_async(self.handle, int(n)))

    def sync(self) -> int:
        rc = _check(load().sse_batch_sync(self.handle), allow=(SSE_ENONFINITE,))
        self._retired.clear()
        return rc

    def query(self) -> bool:
        """True once the steps enqueued on the batch's stream have finished
        (does not wait; ``sync`` then returns at once with their status)."""
        import torch
        s = self.stream if self.stream is not None else torch.cuda.current_stream()
        return bool(s.query())

    def close(self):
        if self.handle:
            load().sse_batch_destroy(self.handle)
            self.handle = c_void_p()
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
