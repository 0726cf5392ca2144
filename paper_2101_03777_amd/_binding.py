"""ctypes binding of libcrhyb.so (include/crhyb.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module converts numpy /
torch arguments to pointers and status codes to exceptions.  If the built
library is missing, load() raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrhyb.so")

CR_OK, CR_E_INVAL, CR_E_NOMEM, CR_E_MESH, CR_E_SINGULAR, CR_E_NOCONV, CR_E_BREAKDOWN, CR_E_NONFINITE, CR_E_DEVICE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {0: "CR_OK", -1: "CR_E_INVAL", -2: "CR_E_NOMEM", -3: "CR_E_MESH", -4: "CR_E_SINGULAR",
                -5: "CR_E_NOCONV", -6: "CR_E_BREAKDOWN", -7: "CR_E_NONFINITE", -8: "CR_E_DEVICE"}
CR_STOKES, CR_NS_NEWTON = 0, 1
CR_RCM, CR_NATURAL = 0, 1
CR_PCG, CR_BICGSTAB, CR_BICGSTAB2, CR_MINRES = 0, 1, 2, 3
CR_FP64, CR_FP32_IR = 0, 1
CR_OP_AUTO, CR_OP_ASSEMBLED, CR_OP_ELEMENT = 0, 1, 2
_OPFORM = {"auto": CR_OP_AUTO, "assembled": CR_OP_ASSEMBLED, "element": CR_OP_ELEMENT}
CR_PC_DEFAULT, CR_PC_JACOBI, CR_PC_COARSE = 0, 1, 2
_PRECOND = {"default": CR_PC_DEFAULT, "jacobi": CR_PC_JACOBI, "coarse": CR_PC_COARSE}

# every function declared in include/crhyb.h
EXPORTS = ["cr_assemble", "cr_eliminate", "cr_update_rhs", "cr_solve", "cr_recover", "cr_query_sizes",
           "cr_export_G", "cr_export_W", "cr_export_W_device", "cr_import_W", "cr_interior_faces", "cr_topology", "cr_coupled_solve",
           "cr_time_spmv", "cr_destroy", "cr_last_error", "cr_version", "cr_batch_create", "cr_batch_add",
           "cr_batch_advance", "cr_batch_pop", "cr_batch_count", "cr_batch_destroy", "cr_prepare",
           "cr_assemble_prepared", "cr_prepared_destroy", "cr_export_coupled", "cr_recover_noalloc",
           "cr_boundary_faces", "cr_set_boundary"]


class CRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64), ("coords", C.POINTER(C.c_double)),
                ("n_elements", C.c_int64), ("elem_vertices", C.POINTER(C.c_int32))]


class Params(C.Structure):
    _fields_ = [("mu", C.c_double), ("nu", C.c_double), ("k0", C.c_int32), ("problem", C.c_int32),
                ("renumber", C.c_int32), ("lambda_scale", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("maxit", C.c_int32), ("max_outer", C.c_int32), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("warm_start", C.c_int32), ("operator_form", C.c_int32),
                ("precond", C.c_int32), ("w0", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("rel_residual", C.c_double),
                ("t_solve_ms", C.c_double), ("reason", C.c_int32), ("fp32_iters", C.c_int32),
                ("fp64_fallback", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the built HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or "
                           "python -m paper_2101_03777_amd.build")
    # torch first: its HIP runtime then provides the library's HIP symbols, so
    # the process holds one runtime (device pointers and streams come from
    # torch).  Loaded the other way round, the library would bring in a second
    # HIP runtime, and device calls through one of them can fail.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "cr_assemble": (I32, [C.POINTER(MeshDesc), C.POINTER(Params), C.POINTER(Allocator), P, C.POINTER(P)]),
        "cr_eliminate": (I32, [P, P, P, P]),
        "cr_update_rhs": (I32, [P, P, P]),
        "cr_solve": (I32, [P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
        "cr_recover": (I32, [P, P, P, P]),
        "cr_recover_noalloc": (I32, [P, P, P, P]),
        "cr_query_sizes": (I32, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
        "cr_export_G": (I32, [P, P, P, P, P]),
        "cr_export_W": (I32, [P, P]),
        "cr_export_W_device": (I32, [P, P]),
        "cr_export_coupled": (I32, [P, P, P, P, P]),
        "cr_import_W": (I32, [P, P]),
        "cr_interior_faces": (I32, [P, P]),
        "cr_boundary_faces": (I32, [P, C.POINTER(I64), P]),
        "cr_set_boundary": (I32, [P, P]),
        "cr_topology": (I32, [C.POINTER(MeshDesc), C.POINTER(Params), C.POINTER(I64), P, C.POINTER(I64),
                              C.POINTER(I64), P]),
        "cr_coupled_solve": (I32, [P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), P, P]),
        "cr_time_spmv": (I32, [P, I32, I32, I32, C.POINTER(D), C.POINTER(D)]),
        "cr_destroy": (None, [P]),
        "cr_prepare": (I32, [C.POINTER(MeshDesc), C.POINTER(Params), C.POINTER(P)]),
        "cr_assemble_prepared": (I32, [P, C.POINTER(Allocator), P, C.POINTER(P)]),
        "cr_prepared_destroy": (None, [P]),
        "cr_batch_create": (I32, [P, I32, C.POINTER(P)]),
        "cr_batch_add": (I32, [P, P, C.POINTER(SolveOpts)]),
        "cr_batch_advance": (I32, [P, I32, C.POINTER(I32)]),
        "cr_batch_pop": (I32, [P, C.POINTER(P), C.POINTER(SolveInfo), C.POINTER(I32)]),
        "cr_batch_count": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
        "cr_batch_destroy": (None, [P]),
        "cr_last_error": (C.c_char_p, []),
        "cr_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != CR_OK:
        raise CRError(status, load().cr_last_error().decode())


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _mesh(coords, elems):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    elems = np.ascontiguousarray(elems, dtype=np.int32)
    m = MeshDesc(coords.shape[1], coords.shape[0], coords.ctypes.data_as(C.POINTER(C.c_double)),
                 elems.shape[0], elems.ctypes.data_as(C.POINTER(C.c_int32)))
    return m, (coords, elems)


def _params(mu, nu, k0, problem, renumber, lambda_scale=0.0):
    prob = {"stokes": CR_STOKES, "ns": CR_NS_NEWTON}[problem] if isinstance(problem, str) else int(problem)
    ren = {"rcm": CR_RCM, "natural": CR_NATURAL}[renumber] if isinstance(renumber, str) else int(renumber)
    return Params(float(mu), float(nu), int(k0), prob, ren, float(lambda_scale))


def topology(coords, elems, mu=1.0, nu=1.0, k0=0, problem="stokes", renumber="rcm"):
    """Host-only step a0 (no device work): face count, internal position of each
    canonical face, bandwidths (internal, canonical) and the M1 flags."""
    lib = load()
    m, keep = _mesh(coords, elems)
    p = _params(mu, nu, k0, problem, renumber)
    nf = C.c_int64()
    _check(lib.cr_topology(C.byref(m), C.byref(p), C.byref(nf), None, None, None, None))
    perm = np.empty(nf.value, dtype=np.int32)
    m1 = np.empty(keep[1].shape[0], dtype=np.int32)
    bwi, bwc = C.c_int64(), C.c_int64()
    _check(lib.cr_topology(C.byref(m), C.byref(p), C.byref(nf), _ptr(perm), C.byref(bwi), C.byref(bwc), _ptr(m1)))
    return dict(n_int_faces=nf.value, perm=perm, bandwidth_internal=bwi.value, bandwidth_canonical=bwc.value,
                m1=m1.astype(bool))


class TorchAllocator:
    """cr_allocator backed by torch's caching allocator, so that device memory is
    accounted by torch (and by a serving loop's memory budget)."""

    def __init__(self, device=0):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self._alloc = ALLOC_FN(self._do_alloc)
        self._release = RELEASE_FN(self._do_release)
        self.struct = Allocator(self._alloc, self._release, None)

    def _do_alloc(self, nbytes, ctx, stream):
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
        except Exception:
            return None
        self.live[p] = int(nbytes)
        return p

    def _do_release(self, ptr, ctx, stream):
        if ptr in self.live:
            del self.live[ptr]
            if not sys.is_finalizing():
                self._torch.cuda.caching_allocator_delete(ptr)

    @property
    def bytes_in_use(self):
        return sum(self.live.values())


METHODS = {"pcg": CR_PCG, "bicgstab": CR_BICGSTAB, "bicgstab2": CR_BICGSTAB2, "minres": CR_MINRES}


def solve_opts(method="pcg", precision="fp32_ir", tol=1e-10, inner_tol=0.0, maxit=0, max_outer=0,
               check_every=0, graph=True, warm_start=False, operator="auto", coarse=True, precond=None, w0=None):
    """cr_solve_opts; precond ("default", "jacobi", "coarse") overrides coarse
    (True: "default", False: "jacobi"); w0 is a device float64 tensor
    [n_int_faces, dim] (canonical) or None."""
    pc = _PRECOND[precond] if precond is not None else (CR_PC_DEFAULT if coarse else CR_PC_JACOBI)
    return SolveOpts(METHODS[method], {"fp64": CR_FP64, "fp32_ir": CR_FP32_IR}[precision], float(tol),
                     float(inner_tol), int(maxit), int(max_outer), int(check_every), int(bool(graph)),
                     int(bool(warm_start)), _OPFORM[operator], pc, None if w0 is None else w0.data_ptr())


def info_dict(st, info):
    return dict(status=st, iters=info.iters, outer_iters=info.outer_iters, rel_residual=info.rel_residual,
                t_solve_ms=info.t_solve_ms, reason=info.reason, fp32_iters=info.fp32_iters,
                fp64_fallback=bool(info.fp64_fallback))


class Batch:
    """Batched CG solves of resident systems (cr_batch_*): shared launches over
    all active systems, each system's iterates identical to a single solve."""

    def __init__(self, max_systems=256, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = C.c_void_p()
        _check(self.lib.cr_batch_create(C.c_void_p(handle), int(max_systems), C.byref(h)))
        self.h = h
        self._members = {}

    def add(self, system, **opts):
        o = solve_opts(**opts)
        _check(self.lib.cr_batch_add(self.h, system.h, C.byref(o)))
        self._members[system.h.value] = system

    def advance(self, n_iters=32):
        n = C.c_int32()
        _check(self.lib.cr_batch_advance(self.h, int(n_iters), C.byref(n)))
        return n.value

    def pop(self):
        """Next finished (system, info dict) or None."""
        p = C.c_void_p()
        info = SolveInfo()
        st = C.c_int32()
        _check(self.lib.cr_batch_pop(self.h, C.byref(p), C.byref(info), C.byref(st)))
        if not p.value:
            return None
        return self._members.pop(p.value), info_dict(st.value, info)

    def count(self):
        a, f = C.c_int32(), C.c_int32()
        _check(self.lib.cr_batch_count(self.h, C.byref(a), C.byref(f)))
        return a.value, f.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.cr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Prepared:
    """Host part of a system (cr_prepare): topology and tables, no device call,
    so it can be built on a worker thread while the device is busy.  Pass it to
    System(prepared=...), which consumes it."""

    def __init__(self, coords, elems, mu, nu, k0=0, problem="stokes", renumber="rcm", lambda_scale=0.0):
        self.lib = load()
        self.dim = int(np.asarray(coords).shape[1])
        self.n_elements = int(np.asarray(elems).shape[0])
        m, keep = _mesh(coords, elems)
        p = _params(mu, nu, k0, problem, renumber, lambda_scale)
        h = C.c_void_p()
        _check(self.lib.cr_prepare(C.byref(m), C.byref(p), C.byref(h)))
        self.h = h

    def take(self):
        h, self.h = self.h, None
        if h is None:
            raise ValueError("prepared mesh already assembled")
        return h

    def __del__(self):
        if getattr(self, "h", None) is not None and not sys.is_finalizing():
            self.lib.cr_prepared_destroy(self.h)
            self.h = None


class System:
    """One hybridised Crouzeix-Raviart system resident on the current GPU."""

    def __init__(self, coords=None, elems=None, mu=None, nu=None, k0=0, problem="stokes", renumber="rcm",
                 stream=None, allocator="torch", prepared=None, lambda_scale=0.0):
        import torch
        self._torch = torch
        self.lib = load()
        if prepared is not None:
            self.dim, self.n_elements = prepared.dim, prepared.n_elements
        else:
            self.dim = int(np.asarray(coords).shape[1])
            self.n_elements = int(np.asarray(elems).shape[0])
        self.device = torch.cuda.current_device()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._alloc = TorchAllocator(self.device) if allocator == "torch" else None
        h = C.c_void_p()
        al = C.byref(self._alloc.struct) if self._alloc else None
        if prepared is not None:
            _check(self.lib.cr_assemble_prepared(prepared.take(), al, C.c_void_p(handle), C.byref(h)))
        else:
            m, keep = _mesh(coords, elems)
            p = _params(mu, nu, k0, problem, renumber, lambda_scale)
            _check(self.lib.cr_assemble(C.byref(m), C.byref(p), al, C.c_void_p(handle), C.byref(h)))
        self.h = h
        nf, ng, nc = C.c_int64(), C.c_int64(), C.c_int64()
        _check(self.lib.cr_query_sizes(h, C.byref(nf), C.byref(ng), C.byref(nc)))
        self.n_int_faces, self.nnz_G, self.nnz_coupled = nf.value, ng.value, nc.value

    # -- inputs must be device float64 tensors, contiguous -------------------
    def _dev(self, t, shape):
        if t is None:
            return None
        torch = self._torch
        if isinstance(t, np.ndarray):
            t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).cuda()
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
        return t

    def eliminate(self, f_mean, u_prev=None, u_lin=None):
        f = self._dev(f_mean, (self.n_elements, self.dim))
        up = self._dev(u_prev, (self.n_int_faces, self.dim))
        ul = self._dev(u_lin, (self.n_int_faces, self.dim))
        self._keep = (f, up, ul)
        _check(self.lib.cr_eliminate(self.h, _ptr(f), _ptr(up), _ptr(ul)))

    def update_rhs(self, f_mean, u_prev=None):
        f = self._dev(f_mean, (self.n_elements, self.dim))
        up = self._dev(u_prev, (self.n_int_faces, self.dim))
        self._keep = (f, up)
        _check(self.lib.cr_update_rhs(self.h, _ptr(f), _ptr(up)))

    def solve(self, method="pcg", precision="fp32_ir", tol=1e-10, inner_tol=0.0, maxit=0, max_outer=0,
              check_every=0, graph=True, warm_start=False, raise_on_error=True, operator="auto", coarse=True,
              precond=None, w0=None):
        w0 = self._dev(w0, (self.n_int_faces, self.dim))
        o = solve_opts(method, precision, tol, inner_tol, maxit, max_outer, check_every, graph, warm_start,
                       operator, coarse, precond, w0)
        info = SolveInfo()
        st = self.lib.cr_solve(self.h, C.byref(o), C.byref(info))
        out = info_dict(st, info)
        if raise_on_error:
            _check(st)
        return out

    def recover(self, jump=False):
        torch = self._torch
        U = torch.empty((self.n_int_faces, self.dim), dtype=torch.float64, device="cuda")
        P = torch.empty((self.n_elements,), dtype=torch.float64, device="cuda")
        J = torch.empty((1,), dtype=torch.float64, device="cuda") if jump else None
        _check(self.lib.cr_recover(self.h, _ptr(U), _ptr(P), _ptr(J)))
        return (U, P, J) if jump else (U, P)

    def recover_noalloc(self, U, P, J=None):
        """cr_recover_noalloc into caller-provided device tensors U [n_int_faces, dim],
        P [n_elements] and J [1] (or None): no device memory is allocated."""
        torch = self._torch
        for t, shape in ((U, (self.n_int_faces, self.dim)), (P, (self.n_elements,)), (J, (1,))):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or tuple(t.shape) != shape):
                raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
        _check(self.lib.cr_recover_noalloc(self.h, _ptr(U), _ptr(P), _ptr(J)))

    def coupled_solve(self, tol=1e-10, maxit=0, check_every=0, raise_on_error=True, method=None):
        """cr_coupled_solve: FP64 Krylov on the coupled system (MINRES for Stokes,
        BiCGStab(2) or method="bicgstab" for the Newton step)."""
        torch = self._torch
        U = torch.empty((self.n_int_faces, self.dim), dtype=torch.float64, device="cuda")
        P = torch.empty((self.n_elements,), dtype=torch.float64, device="cuda")
        m = METHODS[method] if method is not None else 0
        o = SolveOpts(m, CR_FP64, float(tol), 0.0, int(maxit), 1, int(check_every), 0, 0, CR_OP_AUTO, 0, None)
        info = SolveInfo()
        st = self.lib.cr_coupled_solve(self.h, C.byref(o), C.byref(info), _ptr(U), _ptr(P))
        if raise_on_error:
            _check(st)
        return U, P, dict(status=st, iters=info.iters, rel_residual=info.rel_residual,
                          t_solve_ms=info.t_solve_ms, reason=info.reason)

    def export_G(self):
        import scipy.sparse as sps
        n = self.n_int_faces * self.dim
        rowptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(self.nnz_G, dtype=np.int32)
        val = np.empty(self.nnz_G, dtype=np.float64)
        S = np.empty(n, dtype=np.float64)
        _check(self.lib.cr_export_G(self.h, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(S)))
        return sps.csr_matrix((val, col, rowptr), shape=(n, n)), S

    def export_coupled(self):
        """The coupled matrix [A D^t; D 0] (scipy CSR) and [R; 0], Stokes only."""
        import scipy.sparse as sps
        n = self.n_int_faces * self.dim + self.n_elements - 1
        rowptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(self.nnz_coupled, dtype=np.int32)
        val = np.empty(self.nnz_coupled, dtype=np.float64)
        R = np.empty(n, dtype=np.float64)
        _check(self.lib.cr_export_coupled(self.h, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(R)))
        return sps.csr_matrix((val, col, rowptr), shape=(n, n)), R

    def export_W(self):
        W = np.empty((self.n_int_faces, self.dim), dtype=np.float64)
        _check(self.lib.cr_export_W(self.h, _ptr(W)))
        return W

    def export_W_device(self, out=None):
        """The resident W [n_int_faces, dim] (canonical) into a device tensor, on
        the system's stream (no host copy)."""
        torch = self._torch
        if out is None:
            out = torch.empty((self.n_int_faces, self.dim), dtype=torch.float64, device="cuda")
        out = self._dev(out, (self.n_int_faces, self.dim))
        _check(self.lib.cr_export_W_device(self.h, _ptr(out)))
        return out

    def import_W(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(self.n_int_faces, self.dim)
        _check(self.lib.cr_import_W(self.h, _ptr(W)))

    def boundary_faces(self):
        """Exterior faces [n_bnd_faces, dim] (sorted vertex ids), the order of set_boundary's data."""
        n = C.c_int64()
        _check(self.lib.cr_boundary_faces(self.h, C.byref(n), None))
        fv = np.empty((n.value, self.dim), dtype=np.int32)
        _check(self.lib.cr_boundary_faces(self.h, C.byref(n), _ptr(fv)))
        return fv

    def set_boundary(self, g):
        """Non-homogeneous Dirichlet data: face means [n_bnd_faces, dim] (device
        tensor or numpy array), or None for homogeneous data."""
        if g is None:
            _check(self.lib.cr_set_boundary(self.h, None))
            self._gb = None
            return
        torch = self._torch
        if isinstance(g, np.ndarray):
            g = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float64)).cuda()
        n = C.c_int64()
        _check(self.lib.cr_boundary_faces(self.h, C.byref(n), None))
        g = self._dev(g, (n.value, self.dim))
        self._gb = g
        _check(self.lib.cr_set_boundary(self.h, _ptr(g)))

    def interior_faces(self):
        fv = np.empty((self.n_int_faces, self.dim), dtype=np.int32)
        _check(self.lib.cr_interior_faces(self.h, _ptr(fv)))
        return fv

    def time_spmv(self, precision="fp32_ir", reps=50, operator="auto"):
        ms, by = C.c_double(), C.c_double()
        _check(self.lib.cr_time_spmv(self.h, {"fp64": CR_FP64, "fp32_ir": CR_FP32_IR}[precision],
                                     _OPFORM[operator], int(reps), C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.cr_destroy(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the process releases device memory itself
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
