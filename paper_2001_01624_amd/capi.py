"""ctypes binding of ``libmsrsb.so`` (declared in ``include/msrsb.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (the tensors passed to ``solve``, ``apply``,
``fluxes`` and ``add_dynamic_basis``) and the stream.  Importing this module
raises if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsrsb.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_SINGULAR, E_NOCONV, E_STATE = 0, -1, -2, -3, -4, -5, -6
PART_CARTESIAN, PART_GRAPH, PART_FAULT_CUT = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_ILU0_RB, SMOOTH_ILU0_LINE = 0, 1, 2
FP64, MIXED = 0, 1
RICHARDSON, GMRES = 0, 1
OP_RESIDUAL, OP_SMOOTH, OP_PRECOND, OP_MATVEC = 0, 1, 2, 3
NOALLOC_MAX_CELLS = 2097152
K_CLASSES = {"sweep": 1, "residual": 2, "smooth": 3, "restrict": 4, "prolong": 5, "coarse": 6, "ortho": 7,
             "matvec": 8, "rap": 9, "inverse": 10, "restrict_rows": 11}
_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_SINGULAR", -5: "E_NOCONV", -6: "E_STATE"}


class MsrsbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("active", C.POINTER(C.c_uint8)),
                ("tx", C.POINTER(C.c_double)), ("ty", C.POINTER(C.c_double)), ("tz", C.POINTER(C.c_double)),
                ("fault", C.POINTER(C.c_uint8)),
                ("n_bc", C.c_int32), ("bc_cell", C.POINTER(C.c_int32)),
                ("bc_trans", C.POINTER(C.c_double)), ("bc_value", C.POINTER(C.c_double)),
                ("source", C.POINTER(C.c_double))]


class Partition(C.Structure):
    _fields_ = [("kind", C.c_int32), ("coarse_dims", C.c_int32 * 3), ("parent", C.c_int32),
                ("block_of_cell", C.POINTER(C.c_int32)), ("overlap", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("omega", C.c_double), ("omega_s", C.c_double), ("smoother", C.c_int32),
                ("precision", C.c_int32), ("n_bins", C.c_int32), ("max_dyn_blocks", C.c_int32),
                ("outer", C.c_int32), ("restart", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


def torch_allocator(device):
    """An ``msrsb_allocator`` backed by PyTorch's caching allocator on
    ``device``: blocks are taken on the context's stream and returned to the
    cache (``caching_allocator_alloc`` / ``caching_allocator_delete``)."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=int(stream or 0))
        except Exception:  # out of memory or a bad stream: the library reports E_NOMEM
            return None

    def _free(ptr, nbytes, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    a = Allocator()
    a.alloc, a.free, a.user = _ALLOC_FN(_alloc), _FREE_FN(_free), None
    return a


class Fluid(C.Structure):
    _fields_ = [("mu_w", C.c_double), ("mu_o", C.c_double), ("n_w", C.c_double), ("n_o", C.c_double)]


def _load():
    # PyTorch ships its own HIP runtime (same soname as the system one).  Load
    # it first so that the library binds to that runtime: one runtime per
    # process, and torch's streams and allocations are valid handles here.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2001_01624_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, I, D, VP = C.POINTER, C.c_int, C.c_double, C.c_void_p
    sig = {
        "msrsb_last_error": (C.c_char_p, []),
        "msrsb_default_options": (None, [P(Options)]),
        "msrsb_footprint_bytes": (C.c_size_t, [P(Grid), I, P(Partition), P(Options)]),
        "msrsb_setup": (I, [P(Grid), I, P(Partition), P(Options), P(Allocator), VP, P(VP)]),
        "msrsb_update_basis": (I, [VP, I, P(D), P(D), I, D, I, P(I), P(D)]),
        "msrsb_add_dynamic_basis": (I, [VP, I, P(VP), P(I)]),
        "msrsb_clear_dynamic_basis": (I, [VP]),
        "msrsb_solve": (I, [VP, VP, VP, D, I, P(I), P(D)]),
        "msrsb_solve_async": (I, [VP, VP, VP, D, I, VP]),
        "msrsb_faces_to_box": (I, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(C.c_int32), P(D), P(D), P(D),
                                   P(D)]),
        "msrsb_apply": (I, [VP, I, VP, VP]),
        "msrsb_solve_fv": (I, [VP, I, VP, VP, VP, VP, VP, D, I, P(I), P(D)]),
        "msrsb_fluxes": (I, [VP, VP, VP, VP]),
        "msrsb_num_stages": (I, [VP]),
        "msrsb_stage_info": (I, [VP, I, P(I), P(I), P(I)]),
        "msrsb_export_stage": (I, [VP, I, P(C.c_int32), P(C.c_int32), P(D), P(D)]),
        "msrsb_export_stage_noalloc": (I, [VP, I, P(C.c_int32), P(C.c_int32), P(D), P(D)]),
        "msrsb_coarse_apply": (I, [VP, I, P(D), P(D)]),
        "msrsb_set_stream": (I, [VP, VP]),
        "msrsb_destroy": (None, [VP]),
        "msrsb_validate_grid": (I, [P(Grid)]),
        "msrsb_axis_support": (I, [I, I, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)]),
        "msrsb_partition_wells": (I, [P(Grid), I, P(C.c_int32), P(C.c_int32), I, P(C.c_int32)]),
        "msrsb_partition_indicator": (I, [P(Grid), P(D), I, P(C.c_int32), I, P(C.c_int32)]),
        "msrsb_tp_create": (I, [VP, P(D), P(Fluid), I, P(VP)]),
        "msrsb_tp_assemble": (I, [VP, D, VP, VP, VP, VP, I, VP, P(D)]),
        "msrsb_tp_apply": (I, [VP, I, VP, VP]),
        "msrsb_tp_solve": (I, [VP, VP, D, I, P(I), P(D)]),
        "msrsb_tp_update": (I, [VP, VP, VP, VP]),
        "msrsb_tp_destroy": (None, [VP]),
        "msrsb_batch_create": (I, [I, P(VP), VP, P(VP)]),
        "msrsb_batch_update_basis": (I, [VP, I, D, P(C.c_int32)]),
        "msrsb_batch_solve": (I, [VP, P(VP), P(VP), D, I, P(C.c_int32), P(D), P(C.c_int32)]),
        "msrsb_batch_destroy": (None, [VP]),
        "msrsb_profile_begin": (I, [VP, I, I]),
        "msrsb_profile_end": (I, [VP, P(D), P(I)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib, list(sig)


_lib, EXPORTED = _load()


def last_error() -> str:
    return (_lib.msrsb_last_error() or b"").decode()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise MsrsbError(rc, last_error())
    return rc


def default_options(**kw) -> Options:
    o = Options()
    _lib.msrsb_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "smoother" and isinstance(v, str):
            v = {"jacobi": SMOOTH_JACOBI, "ilu0_rb": SMOOTH_ILU0_RB, "ilu0_line": SMOOTH_ILU0_LINE}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "mixed": MIXED}[v]
        if k == "outer" and isinstance(v, str):
            v = {"richardson": RICHARDSON, "gmres": GMRES}[v]
        setattr(o, k, v)
    return o


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


class _GridArrays:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, prob):
        nx, ny, nz = prob.dims
        self.active = np.ascontiguousarray(prob.active, dtype=np.uint8)
        self.tx = np.ascontiguousarray(prob.tx, dtype=np.float64)
        self.ty = np.ascontiguousarray(prob.ty, dtype=np.float64)
        self.tz = np.ascontiguousarray(prob.tz, dtype=np.float64)
        fault = getattr(prob, "fault", None)
        self.fault = None if fault is None else np.ascontiguousarray(fault, dtype=np.uint8).reshape(-1)
        self.bc_cell = np.ascontiguousarray(prob.bc_cell, dtype=np.int32)
        self.bc_trans = np.ascontiguousarray(prob.bc_trans, dtype=np.float64)
        self.bc_value = np.ascontiguousarray(prob.bc_value, dtype=np.float64)
        self.source = np.ascontiguousarray(prob.source, dtype=np.float64)
        g = Grid()
        g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
        g.active = _ptr(self.active, C.c_uint8)
        g.tx, g.ty, g.tz = _ptr(self.tx, C.c_double), _ptr(self.ty, C.c_double), _ptr(self.tz, C.c_double)
        g.fault = _ptr(self.fault, C.c_uint8)
        g.n_bc = int(self.bc_cell.size)
        g.bc_cell = _ptr(self.bc_cell, C.c_int32)
        g.bc_trans = _ptr(self.bc_trans, C.c_double)
        g.bc_value = _ptr(self.bc_value, C.c_double)
        g.source = _ptr(self.source, C.c_double)
        self.grid = g


class _Parts:
    """Partition structs plus the block vectors they point into (kept alive
    for the duration of the call)."""

    def __init__(self, partitions):
        self.arr = (Partition * len(partitions))()
        self.keep = []
        for k, p in enumerate(partitions):
            kind = p.get("kind", "cartesian")
            self.arr[k].kind = {"cartesian": PART_CARTESIAN, "graph": PART_GRAPH,
                                "fault_cut": PART_FAULT_CUT}.get(kind, kind)
            cd = p.get("coarse_dims", (1, 1, 1))
            self.arr[k].coarse_dims[0], self.arr[k].coarse_dims[1], self.arr[k].coarse_dims[2] = (int(x) for x in cd)
            self.arr[k].parent = int(p.get("parent", 0))
            if p.get("block_of_cell") is not None:
                b = np.ascontiguousarray(p["block_of_cell"], dtype=np.int32)
                self.keep.append(b)
                self.arr[k].block_of_cell = _ptr(b, C.c_int32)
            self.arr[k].overlap = int(p.get("overlap", 0))

    def __len__(self):
        return len(self.arr)


def _parts(partitions):
    return _Parts(partitions)


def validate_grid(prob) -> int:
    ga = _GridArrays(prob)
    return _lib.msrsb_validate_grid(C.byref(ga.grid))


def axis_support(n: int, m: int):
    lo = np.zeros(n, np.int32)
    nv = np.zeros(n, np.int32)
    slo = np.zeros(m, np.int32)
    shi = np.zeros(m, np.int32)
    _check(_lib.msrsb_axis_support(n, m, _ptr(lo, C.c_int32), _ptr(nv, C.c_int32), _ptr(slo, C.c_int32),
                                   _ptr(shi, C.c_int32)))
    return lo, nv, slo, shi


def faces_to_box(dims, face_cells, face_trans):
    """Structured face arrays ``(tx, ty, tz)`` of an ``nx x ny x nz`` box from
    a face list (``msrsb_faces_to_box``): ``face_cells`` [F, 2] ascending
    pairs of box neighbours, ``face_trans`` [F]."""
    nx, ny, nz = (int(d) for d in dims)
    fc = np.ascontiguousarray(face_cells, dtype=np.int32).reshape(-1)
    ft = np.ascontiguousarray(face_trans, dtype=np.float64)
    if fc.size != 2 * ft.size:
        raise MsrsbError(E_INVAL, "face_cells must hold two cells per face")
    n = nx * ny * nz
    t = [np.empty(n, np.float64) for _ in range(3)]
    _check(_lib.msrsb_faces_to_box(nx, ny, nz, ft.size, _ptr(fc, C.c_int32), _ptr(ft, C.c_double),
                                   *(_ptr(a, C.c_double) for a in t)))
    return t[0], t[1], t[2]


def partition_wells(prob, wells, radius=0):
    """Well partition (``msrsb_partition_wells``): ``wells`` is a list of
    arrays of box cell indices; returns the block per cell (-1 inactive)."""
    ga = _GridArrays(prob)
    ptr = np.zeros(len(wells) + 1, np.int32)
    ptr[1:] = np.cumsum([len(w) for w in wells])
    cells = np.ascontiguousarray(np.concatenate([np.asarray(w) for w in wells]), dtype=np.int32)
    out = np.zeros(int(np.prod(prob.dims)), np.int32)
    _check(_lib.msrsb_partition_wells(C.byref(ga.grid), len(wells), _ptr(ptr, C.c_int32), _ptr(cells, C.c_int32),
                                      int(radius), _ptr(out, C.c_int32)))
    return out


def partition_indicator(prob, indicator, n_bins, coarse_dims, min_cells):
    """Indicator agglomeration (``msrsb_partition_indicator``); returns the
    block per cell (-1 inactive)."""
    ga = _GridArrays(prob)
    ind = np.ascontiguousarray(indicator, dtype=np.float64)
    cd = np.ascontiguousarray(coarse_dims, dtype=np.int32)
    out = np.zeros(int(np.prod(prob.dims)), np.int32)
    _check(_lib.msrsb_partition_indicator(C.byref(ga.grid), _ptr(ind, C.c_double), int(n_bins), _ptr(cd, C.c_int32),
                                          int(min_cells), _ptr(out, C.c_int32)))
    return out


def footprint_bytes(prob, partitions, options=None) -> int:
    ga = _GridArrays(prob)
    parts = _parts(partitions)
    o = options if options is not None else default_options()
    return int(_lib.msrsb_footprint_bytes(C.byref(ga.grid), len(partitions), parts.arr, C.byref(o)))


def _dptr(t, n=None, device=None, dtype="float64"):
    """Device address of a contiguous tensor of ``n`` elements on ``device``;
    anything else is rejected before a kernel could read or write past it."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == f"torch.{dtype}"):
        raise MsrsbError(E_INVAL, f"expected a contiguous {dtype} device tensor")
    if n is not None and t.numel() != n:
        raise MsrsbError(E_INVAL, f"expected {n} entries, got {t.numel()}")
    if device is not None and t.device.index != device:
        raise MsrsbError(E_INVAL, f"tensor on cuda:{t.device.index}, the context lives on cuda:{device}")
    return C.c_void_p(t.data_ptr())


class Solver:
    """One problem on the device (``msrsb_setup`` ... ``msrsb_destroy``)."""

    def __init__(self, prob, partitions, options=None, stream=None, allocator=None):
        """``allocator``: None for the library's own stream-ordered pool, or
        "torch" for PyTorch's caching allocator (``msrsb_allocator``)."""
        import torch

        self.prob_dims = tuple(prob.dims)
        self.N = int(np.prod(prob.dims))
        self.n_bc = int(np.asarray(prob.bc_cell).size)
        self.options = options if options is not None else default_options()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
        ga = _GridArrays(prob)
        parts = _parts(partitions)
        h = C.c_void_p()
        # the callbacks must outlive the context
        self._alloc = torch_allocator(self.device) if allocator == "torch" else None
        if allocator not in (None, "torch"):
            raise MsrsbError(E_INVAL, f"unknown allocator {allocator!r}")
        _check(_lib.msrsb_setup(C.byref(ga.grid), len(partitions), parts.arr, C.byref(self.options),
                                C.byref(self._alloc) if self._alloc is not None else None,
                                C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def _vec(self, t):
        """A per-cell device vector of this context ([N] float64 on its device)."""
        return _dptr(t, n=self.N, device=self.device)

    def close(self):
        # two-phase contexts borrow this one: they go first
        for dep in list(getattr(self, "_dependents", ())):
            dep.close()
        if getattr(self, "h", None):
            _lib.msrsb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_basis(self, stage=-1, max_sweeps=100, tol=1e-3, warm=False, new_trans=None, new_bc_trans=None):
        """``new_trans``: optional ``(tx, ty, tz)`` host arrays replacing the
        face transmissibilities before the sweeps; ``new_bc_trans``: optional
        connection coefficients (``n_bc``)."""
        sw = C.c_int(0)
        ch = C.c_double(0.0)
        T = None
        if new_trans is not None:
            T = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64).reshape(-1) for t in new_trans]))
            if T.size != 3 * self.N:
                raise MsrsbError(E_INVAL, f"expected 3 x {self.N} transmissibilities, got {T.size}")
        B = None
        if new_bc_trans is not None:
            B = np.ascontiguousarray(new_bc_trans, dtype=np.float64).reshape(-1)
            if B.size != self.n_bc:
                raise MsrsbError(E_INVAL, f"expected {self.n_bc} connection coefficients, got {B.size}")
        _check(_lib.msrsb_update_basis(self.h, stage, _ptr(T, C.c_double), _ptr(B, C.c_double), max_sweeps, tol,
                                       int(warm), C.byref(sw), C.byref(ch)))
        return sw.value, ch.value

    def add_dynamic_basis(self, increments):
        ptrs = (C.c_void_p * len(increments))(*[self._vec(t).value for t in increments])
        counts = (C.c_int * len(increments))()
        _check(_lib.msrsb_add_dynamic_basis(self.h, len(increments), ptrs, counts))
        return list(counts)

    def clear_dynamic_basis(self):
        _check(_lib.msrsb_clear_dynamic_basis(self.h))

    def solve(self, p, source=None, rtol=1e-6, max_iters=500):
        """Solve in place on the device tensor ``p``; returns (iters, relres, status)."""
        it = C.c_int(0)
        rel = C.c_double(0.0)
        rc = _check(_lib.msrsb_solve(self.h, self._vec(source), self._vec(p), rtol, max_iters, C.byref(it),
                                     C.byref(rel)),
                    allow=(E_NOCONV,))
        return it.value, rel.value, rc

    def solve_async(self, p, source=None, rtol=1e-6, max_cycles=200, result=None):
        """Enqueue Richardson cycles on the context's stream without waiting
        (``msrsb_solve_async``).  ``result`` (a 16-byte uint8 device tensor,
        allocated when None) receives status, cycles and relative residual;
        read them with ``read_result`` after synchronising the stream."""
        import torch

        if result is None:
            result = torch.zeros(16, dtype=torch.uint8, device=torch.device("cuda", self.device))
        if result.dtype != torch.uint8 or result.numel() < 16 or not result.is_contiguous():
            raise MsrsbError(E_INVAL, "result must be a contiguous device tensor of 16 bytes")
        _check(_lib.msrsb_solve_async(self.h, self._vec(source), self._vec(p), float(rtol), int(max_cycles),
                                      C.c_void_p(result.data_ptr())))
        return result

    @staticmethod
    def read_result(result):
        """(status, cycles, relres) from a result tensor of ``solve_async``."""
        b = result.cpu().numpy().tobytes()
        st, cyc = np.frombuffer(b[:8], dtype=np.int32)
        return int(st), int(cyc), float(np.frombuffer(b[8:16], dtype=np.float64)[0])

    def solve_fv(self, stage=0, source=None, local_rtol=1e-12, max_local_iters=5000, fine=True):
        """Finite-volume multiscale pressure of one stage and conservative
        fluxes (``msrsb_solve_fv``).  Returns ``(p_ms, p_fine, face[3, N],
        bc_flux, local_iters, max_imbalance)`` as device tensors and floats."""
        import torch

        dev = torch.device("cuda", self.device)
        p = torch.empty(self.N, dtype=torch.float64, device=dev)
        pf = torch.empty(self.N, dtype=torch.float64, device=dev) if fine else None
        face = torch.empty(3 * self.N, dtype=torch.float64, device=dev)
        bcf = torch.empty(max(self.n_bc, 1), dtype=torch.float64, device=dev)
        its = C.c_int(0)
        imb = C.c_double(0.0)
        _check(_lib.msrsb_solve_fv(self.h, int(stage), self._vec(source), self._vec(p), self._vec(pf), _dptr(face),
                                   _dptr(bcf), float(local_rtol), int(max_local_iters), C.byref(its), C.byref(imb)))
        return p, pf, face.view(3, self.N), bcf[: self.n_bc], its.value, imb.value

    def apply(self, op, x, out=None):
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(_lib.msrsb_apply(self.h, op, self._vec(x), self._vec(out)))
        return out

    def fluxes(self, p):
        import torch

        face = torch.empty(3 * self.N, dtype=torch.float64, device=p.device)
        bcf = torch.empty(max(self.n_bc, 1), dtype=torch.float64, device=p.device)
        _check(_lib.msrsb_fluxes(self.h, self._vec(p), _dptr(face), _dptr(bcf)))
        return face.view(3, self.N), bcf[: self.n_bc]

    def profile_begin(self, kernel_class, max_launches=100000):
        cls = K_CLASSES.get(kernel_class, kernel_class)
        _check(_lib.msrsb_profile_begin(self.h, int(cls), int(max_launches)))

    def profile_end(self):
        """Returns (total kernel milliseconds, launches timed)."""
        ms = C.c_double(0.0)
        n = C.c_int(0)
        _check(_lib.msrsb_profile_end(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def num_stages(self):
        return _lib.msrsb_num_stages(self.h)

    def stage_info(self, k):
        M, kind, ns = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.msrsb_stage_info(self.h, k, C.byref(M), C.byref(kind), C.byref(ns)))
        return M.value, kind.value, ns.value

    def export_stage(self, k, values=True, coarse=True, noalloc=False):
        """Stage k as host arrays; ``noalloc`` uses ``msrsb_export_stage_noalloc``."""
        M, kind, ns = self.stage_info(k)
        block = np.zeros(self.N, np.int32)
        slots = np.zeros(ns * self.N, np.int32)
        vals = np.zeros(ns * self.N) if values else None
        Ac = np.zeros(M * M) if coarse else None
        fn = _lib.msrsb_export_stage_noalloc if noalloc else _lib.msrsb_export_stage
        _check(fn(self.h, k, _ptr(block, C.c_int32), _ptr(slots, C.c_int32), _ptr(vals, C.c_double),
                  _ptr(Ac, C.c_double)))
        out = {"M": M, "kind": kind, "n_slots": ns, "block": block, "slot_block": slots.reshape(ns, self.N)}
        if values:
            out["values"] = vals.reshape(ns, self.N)
        if coarse:
            out["Ac"] = Ac.reshape(M, M)
        return out

    def coarse_apply(self, k, d):
        """``A_c^{-1} d`` by stage k's coarse solve (host vectors of M entries)."""
        M, _, _ = self.stage_info(k)
        d = np.ascontiguousarray(d, dtype=np.float64)
        if d.size != M:
            raise MsrsbError(E_INVAL, f"expected {M} entries, got {d.size}")
        out = np.zeros(M)
        _check(_lib.msrsb_coarse_apply(self.h, k, _ptr(d, C.c_double), _ptr(out, C.c_double)))
        return out

    def dense_basis(self, k):
        """``N x M`` dense basis of stage k (tests / inspection)."""
        e = self.export_stage(k, coarse=False)
        P = np.zeros((self.N, e["M"]))
        for s in range(e["n_slots"]):
            blk = e["slot_block"][s]
            m = blk >= 0
            P[np.nonzero(m)[0], blk[m]] += e["values"][s][m]
        return P


class Batch:
    """Ensemble batch over several ``Solver`` contexts (``msrsb_batch_*``):
    one launch per kernel over all members; each member's results are those
    of its own ``update_basis`` / ``solve``, bit for bit.  The members are
    borrowed (they must outlive the batch) and run on ``stream``."""

    def __init__(self, solvers, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.members = list(solvers)
        n = len(self.members)
        arr = (C.c_void_p * n)(*[s.h.value for s in self.members])
        h = C.c_void_p()
        _check(_lib.msrsb_batch_create(n, arr, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        for s in self.members:
            s.stream = stream

    def update_basis(self, max_sweeps=100, tol=1e-3):
        """Cold basis of every member; returns the sweeps each took."""
        n = len(self.members)
        sw = (C.c_int32 * n)()
        _check(_lib.msrsb_batch_update_basis(self.h, max_sweeps, tol, sw))
        return list(sw)

    def solve(self, ps, sources=None, rtol=1e-6, max_iters=500):
        """Solve every member in place on its device tensor ``ps[k]`` (source
        ``sources[k]``, None keeps the member's source); returns lists of
        (iters, relres, status)."""
        n = len(self.members)
        if len(ps) != n or (sources is not None and len(sources) != n):
            raise MsrsbError(E_INVAL, f"expected {n} vectors")
        pp = (C.c_void_p * n)(*[m._vec(p).value for m, p in zip(self.members, ps)])
        ss = None
        if sources is not None:
            ss = (C.c_void_p * n)(*[(m._vec(q).value if q is not None else None)
                                    for m, q in zip(self.members, sources)])
        it = (C.c_int32 * n)()
        rel = (C.c_double * n)()
        st = (C.c_int32 * n)()
        _check(_lib.msrsb_batch_solve(self.h, ss, pp, rtol, max_iters, it, rel, st), allow=(E_NOCONV,))
        return list(it), list(rel), list(st)

    def close(self):
        if getattr(self, "h", None):
            _lib.msrsb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TwoPhase:
    """Two-phase CPR solver on a pressure ``Solver`` (``msrsb_tp_*``): the
    Jacobian and residual of the water/oil model, the two-stage
    preconditioner and GMRES on the full system.  State vectors are device
    tensors of the pressure context's size; full-system vectors interleave
    (water/pressure, oil/saturation) per cell."""

    OP_MATVEC, OP_CPR = 0, 1

    def __init__(self, solver, pore_volume, fluid, restart=30):
        self.ms = solver
        self.N = solver.N
        f = Fluid(float(fluid["mu_w"]), float(fluid["mu_o"]), float(fluid["n_w"]), float(fluid["n_o"]))
        pv = np.ascontiguousarray(pore_volume, dtype=np.float64)
        if pv.size != self.N:
            raise MsrsbError(E_INVAL, f"expected {self.N} pore volumes, got {pv.size}")
        h = C.c_void_p()
        _check(_lib.msrsb_tp_create(solver.h, _ptr(pv, C.c_double), C.byref(f), int(restart), C.byref(h)))
        self.h = h
        import weakref

        if not hasattr(solver, "_dependents"):
            solver._dependents = weakref.WeakSet()
        solver._dependents.add(self)

    def _vec2(self, t):
        return _dptr(t, n=2 * self.N, device=self.ms.device)

    def assemble(self, dt, p, s, s_old, q=None, basis_sweeps=3, res=None):
        """Returns ``||R||_2``; ``res`` (a [2N] device tensor) receives R."""
        nr = C.c_double(0.0)
        _check(_lib.msrsb_tp_assemble(self.h, float(dt), self.ms._vec(p), self.ms._vec(s), self.ms._vec(s_old),
                                      self.ms._vec(q), int(basis_sweeps), self._vec2(res), C.byref(nr)))
        return nr.value

    def apply(self, op, x, out=None):
        import torch

        if out is None:
            out = torch.empty_like(x)
        _check(_lib.msrsb_tp_apply(self.h, int(op), self._vec2(x), self._vec2(out)))
        return out

    def solve(self, rtol=1e-8, max_iters=500, dx=None):
        """GMRES + CPR on ``J dx = -R``; returns ``(dx, iterations, relres, status)``."""
        import torch

        if dx is None:
            dx = torch.empty(2 * self.N, dtype=torch.float64, device=torch.device("cuda", self.ms.device))
        it = C.c_int(0)
        rel = C.c_double(0.0)
        rc = _check(_lib.msrsb_tp_solve(self.h, self._vec2(dx), float(rtol), int(max_iters), C.byref(it),
                                        C.byref(rel)), allow=(E_NOCONV,))
        return dx, it.value, rel.value, rc

    def update(self, dx, p, s):
        _check(_lib.msrsb_tp_update(self.h, self._vec2(dx), self.ms._vec(p), self.ms._vec(s)))

    def close(self):
        if getattr(self, "h", None):
            # the pressure context must still exist (its close() closes this first)
            if getattr(self.ms, "h", None):
                _lib.msrsb_tp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
