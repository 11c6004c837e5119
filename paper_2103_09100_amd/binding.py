"""ctypes binding of ``libsbfem.so`` (include/sbfem.h); argument marshalling only.

Every computation of the time loop runs in the library's HIP kernels.  If the
library has not been built this module raises on import: there is no CPU
fallback.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbfem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_09100_amd.build`")

# One HIP runtime per process.  The PyTorch wheel carries its own HIP and HSA runtimes
# whose sonames equal the system ones; loaded after torch, the library binds to torch's
# copy, so streams and device pointers handed over from torch are valid here.  Loaded
# first, it would pull in the system copy and torch would then start a second runtime
# that finds no device.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, EBUSY, ENOTCONV = 0, -1, -2, -3, -4, -5, -6
PROD = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
STATE = {"fp64": 0, "fp32": 1, "kahan32": 2}
ASM = {"atomic": 0, "colour": 1, "tiled": 2}
LOAD_KIND = {"ricker": 0, "triangle": 1, "sine_burst": 2, "table": 3}

EXPORTS = ["sbfem_upload_patterns", "sbfem_destroy_patterns", "sbfem_mesh_footprint", "sbfem_plan_mesh",
           "sbfem_create_mesh_planned", "sbfem_destroy_plan",
           "sbfem_critical_dt", "sbfem_create_mesh", "sbfem_destroy_mesh", "sbfem_step_n", "sbfem_set_graph_steps",
           "sbfem_step_batch", "sbfem_step_batch_noalloc", "sbfem_read_state", "sbfem_write_state", "sbfem_mesh_info",
           "sbfem_profile", "sbfem_profile_read", "sbfem_mesh_layout", "sbfem_set_allocator", "sbfem_eigen_lowest",
           "sbfem_set_probes", "sbfem_read_probes", "sbfem_set_check_interval",
           "sbfem_last_error"]
KERNEL_CLASSES = ("load", "element_8node", "element_larger", "update")


class MeshDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("h0", C.c_double),
        ("conn", C.c_void_p), ("pattern", C.c_void_p), ("orient", C.c_void_p),
        ("level", C.c_void_p), ("material", C.c_void_p),
        ("n_materials", C.c_int32), ("E", C.c_void_p), ("rho", C.c_void_p),
        ("fixed_dof", C.c_void_p),
        ("load_nnz", C.c_int64), ("load_dof", C.c_void_p), ("load_val", C.c_void_p),
        ("load_kind", C.c_int32), ("load_t1", C.c_double), ("load_P0", C.c_double),
        ("load_cycles", C.c_int32),
        ("dt", C.c_double), ("alpha", C.c_double),
        ("prod", C.c_int32), ("state", C.c_int32), ("assembly", C.c_int32),
        ("u0", C.c_void_p), ("v0", C.c_void_p),
        ("tile_nodes", C.c_int32), ("block_threads", C.c_int32), ("block_threads_mixed", C.c_int32),
        ("load_table_n", C.c_int64), ("load_table", C.c_void_p),
    ]


_P = C.c_void_p
_lib.sbfem_upload_patterns.argtypes = [C.POINTER(_P), C.c_int32, _P, _P, _P, _P, _P]
_lib.sbfem_destroy_patterns.argtypes = [_P]
_lib.sbfem_destroy_patterns.restype = None
_lib.sbfem_mesh_footprint.argtypes = [_P, C.POINTER(MeshDesc), C.POINTER(C.c_int64)]
_lib.sbfem_critical_dt.argtypes = [_P, C.POINTER(MeshDesc), C.POINTER(C.c_double)]
_lib.sbfem_create_mesh.argtypes = [C.POINTER(_P), _P, C.POINTER(MeshDesc), _P]
_lib.sbfem_plan_mesh.argtypes = [C.POINTER(_P), _P, C.POINTER(MeshDesc), C.POINTER(C.c_int64)]
_lib.sbfem_create_mesh_planned.argtypes = [C.POINTER(_P), _P, _P]
_lib.sbfem_destroy_plan.argtypes = [_P]
_lib.sbfem_destroy_plan.restype = None
_lib.sbfem_destroy_mesh.argtypes = [_P]
_lib.sbfem_destroy_mesh.restype = None
_lib.sbfem_step_n.argtypes = [_P, C.c_int64, _P]
_lib.sbfem_step_batch.argtypes = [_P, C.c_int32, _P, _P]
_lib.sbfem_step_batch_noalloc.argtypes = [_P, C.c_int32, _P, _P]
_lib.sbfem_set_graph_steps.argtypes = [_P, C.c_int32]
_lib.sbfem_read_state.argtypes = [_P, C.c_int32, _P, C.POINTER(C.c_int64), _P]
_lib.sbfem_write_state.argtypes = [_P, _P, _P, C.c_int64, _P]
_lib.sbfem_mesh_info.argtypes = [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
_lib.sbfem_profile.argtypes = [_P, C.c_int32]
_lib.sbfem_profile_read.argtypes = [_P, _P, _P]
_lib.sbfem_mesh_layout.argtypes = [_P, _P, C.c_int32]
_lib.sbfem_eigen_lowest.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, _P, _P,
                                     C.POINTER(C.c_int32), _P]
_lib.sbfem_set_probes.argtypes = [_P, C.c_int32, _P, C.c_int64, _P]
_lib.sbfem_set_check_interval.argtypes = [_P, C.c_int64]
_lib.sbfem_read_probes.argtypes = [_P, _P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _P]
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_lib.sbfem_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, _P]
_lib.sbfem_last_error.argtypes = []
_lib.sbfem_last_error.restype = C.c_char_p
for _name in EXPORTS:
    if _name not in ("sbfem_destroy_patterns", "sbfem_destroy_mesh", "sbfem_last_error"):
        getattr(_lib, _name).restype = C.c_int


class SbfemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sbfem status {status}: {msg}")
        self.status = status


def _check(status):
    if status != OK:
        raise SbfemError(status, _lib.sbfem_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data


def _stream(stream):
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


def last_error():
    return _lib.sbfem_last_error().decode()


class Patterns:
    """Device copy of a master-cell library (see :func:`library.build_library`)."""

    def __init__(self, lib, stream=None):
        K, m = lib.flat()
        self._keep = (np.ascontiguousarray(lib.ndof, dtype=np.int32), np.ascontiguousarray(K),
                      np.ascontiguousarray(m), np.ascontiguousarray(lib.omega))
        h = _P()
        _check(_lib.sbfem_upload_patterns(C.byref(h), len(lib.ndof), *[_ptr(a) for a in self._keep],
                                          _stream(stream)))
        self.handle = h
        self.library = lib

    def close(self):
        if self.handle:
            _lib.sbfem_destroy_patterns(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc(mesh, pid, orient, conn, dt, prod="fp64", state="fp64", assembly="atomic",
              u0=None, v0=None, tile_nodes=0, block_threads=0, block_threads_mixed=0):
    """Descriptor (plus the arrays it points into) for a canonicalised mesh."""
    keep = dict(
        conn=np.ascontiguousarray(conn, dtype=np.int32),
        pattern=np.ascontiguousarray(pid, dtype=np.uint16),
        orient=np.ascontiguousarray(orient, dtype=np.uint8),
        level=np.ascontiguousarray(mesh.cell_level, dtype=np.uint8),
        material=np.ascontiguousarray(mesh.cell_mat, dtype=np.uint8),
        E=np.ascontiguousarray(mesh.mat_E, dtype=np.float64),
        rho=np.ascontiguousarray(mesh.mat_rho, dtype=np.float64),
        fixed=np.ascontiguousarray(mesh.fixed, dtype=np.uint8),
        load_dof=np.ascontiguousarray(mesh.load_dof, dtype=np.int64),
        load_val=np.ascontiguousarray(mesh.load_val, dtype=np.float64),
        u0=None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64),
        v0=None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64),
        load_table=(np.ascontiguousarray(mesh.load["P"], dtype=np.float64)
                    if mesh.load.get("kind") == "table" else None),
    )
    L = mesh.load
    d = MeshDesc()
    d.n_nodes = mesh.n_nodes
    d.n_cells = mesh.n_cells
    d.h0 = mesh.h0
    d.conn = _ptr(keep["conn"])
    d.pattern = _ptr(keep["pattern"])
    d.orient = _ptr(keep["orient"])
    d.level = _ptr(keep["level"])
    d.material = _ptr(keep["material"])
    d.n_materials = len(keep["E"])
    d.E = _ptr(keep["E"])
    d.rho = _ptr(keep["rho"])
    d.fixed_dof = _ptr(keep["fixed"])
    d.load_nnz = len(keep["load_dof"])
    d.load_dof = _ptr(keep["load_dof"]) if d.load_nnz else None
    d.load_val = _ptr(keep["load_val"]) if d.load_nnz else None
    d.load_kind = LOAD_KIND[L.get("kind", "ricker")]
    d.load_t1 = float(L.get("t1", 1.0))
    d.load_P0 = float(L.get("P0", 1.0))
    d.load_cycles = int(L.get("cycles", 5))
    d.dt = float(dt)
    d.alpha = float(L.get("alpha", 0.0))
    d.prod = PROD[prod]
    d.state = STATE[state]
    d.assembly = ASM[assembly]
    d.u0 = _ptr(keep["u0"])
    d.v0 = _ptr(keep["v0"])
    if keep["load_table"] is not None:
        d.load_table_n = len(keep["load_table"])
        d.load_table = _ptr(keep["load_table"])
    d.tile_nodes = int(tile_nodes)
    d.block_threads = int(block_threads)
    d.block_threads_mixed = int(block_threads_mixed)
    return d, keep


def critical_dt(patterns, desc):
    out = C.c_double()
    _check(_lib.sbfem_critical_dt(patterns.handle, C.byref(desc), C.byref(out)))
    return out.value


def footprint(patterns, desc):
    out = C.c_int64()
    _check(_lib.sbfem_mesh_footprint(patterns.handle, C.byref(desc), C.byref(out)))
    return out.value


class Plan:
    """sbfem_plan_mesh: the host set-up of a mesh and its device footprint, kept until
    Mesh(..., plan=) creates the mesh from it (the descriptor and its arrays stay referenced)."""

    def __init__(self, patterns, desc, keep=None):
        h, b = _P(), C.c_int64()
        _check(_lib.sbfem_plan_mesh(C.byref(h), patterns.handle, C.byref(desc), C.byref(b)))
        self.handle, self.footprint = h, b.value
        self.patterns, self.desc, self.keep = patterns, desc, keep

    def close(self):
        if self.handle:
            _lib.sbfem_destroy_plan(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Mesh:
    """A resident simulation (sbfem_mesh); with `plan` (a Plan of the same patterns and
    descriptor) created by sbfem_create_mesh_planned without repeating the host set-up."""

    def __init__(self, patterns, desc, keep=None, stream=None, plan=None):
        h = _P()
        if plan is not None:
            try:
                _check(_lib.sbfem_create_mesh_planned(C.byref(h), plan.handle, _stream(stream)))
            finally:
                plan.close()
        else:
            _check(_lib.sbfem_create_mesh(C.byref(h), patterns.handle, C.byref(desc), _stream(stream)))
        self.handle = h
        self.patterns = patterns
        self.n_dof = 3 * desc.n_nodes
        self.dt = desc.dt

    def step(self, n, stream=None):
        _check(_lib.sbfem_step_n(self.handle, int(n), _stream(stream)))

    def set_graph_steps(self, steps):
        """Replay whole chunks of `steps` steps from a captured HIP graph (0: launch each step)."""
        _check(_lib.sbfem_set_graph_steps(self.handle, int(steps)))

    def read(self, which=0, stream=None):
        out = np.empty(self.n_dof, dtype=np.float64)
        step = C.c_int64()
        _check(_lib.sbfem_read_state(self.handle, int(which), out.ctypes.data, C.byref(step), _stream(stream)))
        return out, step.value

    def write(self, u, um1, step, stream=None):
        u = np.ascontiguousarray(u, dtype=np.float64)
        um1 = np.ascontiguousarray(um1, dtype=np.float64)
        _check(_lib.sbfem_write_state(self.handle, u.ctypes.data, um1.ctypes.data, int(step), _stream(stream)))

    def info(self):
        b, n, c = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.sbfem_mesh_info(self.handle, C.byref(b), C.byref(n), C.byref(c)))
        return dict(device_bytes=b.value, n_dof=n.value, n_colours=c.value)

    LAYOUT = ("tiles_8node", "tiles_other", "items", "local_nodes", "cell_entries", "tile_nodes",
              "alg_bytes_8node", "alg_bytes_other", "max_local_nodes", "lds_bytes")

    def layout(self):
        v = np.zeros(len(self.LAYOUT), dtype=np.int64)
        _check(_lib.sbfem_mesh_layout(self.handle, v.ctypes.data, len(v)))
        return dict(zip(self.LAYOUT, v.tolist()))

    def profile(self, enable=True):
        _check(_lib.sbfem_profile(self.handle, int(bool(enable))))

    def profile_read(self):
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        _check(_lib.sbfem_profile_read(self.handle, ms.ctypes.data, n.ctypes.data))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def set_check_interval(self, steps):
        """sbfem_set_check_interval: step_n examines the non-finite record every `steps` steps."""
        _check(_lib.sbfem_set_check_interval(self.handle, int(steps)))

    def set_probes(self, dofs, capacity, stream=None):
        """sbfem_set_probes: record u_{n+1} and the acceleration of step n at these dofs."""
        d = np.ascontiguousarray(dofs, dtype=np.int64)
        self._probe_count = len(d)
        _check(_lib.sbfem_set_probes(self.handle, len(d), d.ctypes.data if len(d) else None, int(capacity),
                                     _stream(stream)))

    def read_probes(self, stream=None):
        """sbfem_read_probes: (u, a, first step), u and a of shape (rows, probes)."""
        rows, step0 = C.c_int64(), C.c_int64()
        _check(_lib.sbfem_read_probes(self.handle, None, None, C.byref(rows), C.byref(step0), _stream(stream)))
        n = getattr(self, "_probe_count", 0)
        u = np.zeros((rows.value, n))
        a = np.zeros((rows.value, n))
        if rows.value and n:
            _check(_lib.sbfem_read_probes(self.handle, u.ctypes.data, a.ctypes.data, C.byref(rows), C.byref(step0),
                                          _stream(stream)))
        return u, a, step0.value

    def eigen_lowest(self, k, block=0, degree=0, max_iter=200, tol=1e-9, stream=None):
        """sbfem_eigen_lowest: the k smallest circular frequencies, their relative Ritz residuals
        and the iterations used."""
        w = np.zeros(k)
        r = np.zeros(k)
        it = C.c_int32()
        _check(_lib.sbfem_eigen_lowest(self.handle, int(k), int(block), int(degree), int(max_iter), float(tol),
                                       w.ctypes.data, r.ctypes.data, C.byref(it), _stream(stream)))
        return w, r, it.value

    def close(self):
        if self.handle:
            _lib.sbfem_destroy_mesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(meshes, steps, stream=None):
    arr = (_P * len(meshes))(*[m.handle for m in meshes])
    st = np.ascontiguousarray(steps, dtype=np.int64)
    _check(_lib.sbfem_step_batch(arr, len(meshes), st.ctypes.data, _stream(stream)))


def step_batch_noalloc(meshes, steps, stream=None):
    """sbfem_step_batch_noalloc: the batch's work lists in the library's static device buffer."""
    arr = (_P * len(meshes))(*[m.handle for m in meshes])
    st = np.ascontiguousarray(steps, dtype=np.int64)
    _check(_lib.sbfem_step_batch_noalloc(arr, len(meshes), st.ctypes.data, _stream(stream)))


NOALLOC_SCRATCH_BYTES = 8 << 20


_ALLOCATOR_KEEP = []  # the C callbacks must outlive every object created with them


def set_allocator(alloc=None, release=None):
    """sbfem_set_allocator: alloc(nbytes) -> device address (int, 0 on failure) and
    release(address); both None restores hipMalloc/hipFree."""
    if alloc is None and release is None:
        _check(_lib.sbfem_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        return
    fa = ALLOC_FN(lambda n, user: int(alloc(int(n))) or None)
    fr = RELEASE_FN(lambda p, user: release(int(p)))
    _ALLOCATOR_KEEP.append((fa, fr))
    _check(_lib.sbfem_set_allocator(fa, fr, None))
