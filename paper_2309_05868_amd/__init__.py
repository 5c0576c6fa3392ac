"""rcqr: randomized Householder-Cholesky QR with multisketching on one AMD MI355X (gfx950).

Thin binding over the C ABI in include/rcqr.h (librcqr.so, built in-tree by
``python -m paper_2309_05868_amd.build``).  This module only marshals arguments: every step of
the factorization runs in the library's HIP kernels.  PyTorch provides device memory and the
stream.  There is no CPU fallback: without the built library (or without a GPU) the calls fail.

Method: Higgins, Szyld, Boman, Yamazaki, arXiv 2309.05868, Algorithm 3 (rand_cholQR).
"""

import ctypes
import os
import re

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librcqr.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "rcqr.h")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP, E_RANK, E_CHOL, E_SCRATCH = range(8)
STATIC_WORKSPACE_BYTES = 64 << 20  # RCQR_STATIC_WORKSPACE_BYTES: scratch of rcqr_factor_static per GPU
MAX_N = 128  # largest number of columns the kernels accept
# plan flags (include/rcqr.h): single-precision sketch, BF16 Gaussian product, second Cholesky QR, S1 made at plan time
FLAG_SKETCH_FP32, FLAG_GEMM_BF16, FLAG_REORTH, FLAG_SKETCH_AT_PLAN = 1, 2, 4, 8
METHODS = {"rand_cholqr": 0, "cholqr2": 1, "scholqr3": 2}
FINAL_RECOMPUTE, FINAL_MATERIALIZE = 0, 1

_lib = None

_c_i64, _c_u64, _c_i32, _c_u32, _c_p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p

_SIGNATURES = {
    "rcqr_workspace_bytes": (ctypes.c_size_t, [_c_i64, _c_i64, _c_i64, _c_i64, _c_u32]),
    "rcqr_plan": (_c_i32, [ctypes.POINTER(_c_p), _c_i64, _c_i64, _c_i64, _c_i64, _c_u64, _c_u32, _c_p, ctypes.c_size_t, _c_p]),
    "rcqr_factor": (_c_i32, [_c_p, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64]),
    "rcqr_cholqr2": (_c_i32, [_c_p, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64]),
    "rcqr_scholqr3": (_c_i32, [_c_p, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64]),
    "rcqr_info": (_c_i32, [_c_p, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "rcqr_destroy": (_c_i32, [_c_p]),
    "rcqr_status_string": (ctypes.c_char_p, [_c_i32]),
    "rcqr_set_timing": (_c_i32, [_c_p, _c_i32]),
    "rcqr_phase_times": (_c_i32, [_c_p, ctypes.POINTER(ctypes.c_float), _c_i32, ctypes.POINTER(_c_i32)]),
    "rcqr_phase_name": (ctypes.c_char_p, [_c_i32]),
    "rcqr_sketch_hash": (_c_i32, [_c_p, _c_i64, _c_i64, _c_p, _c_p]),
    "rcqr_gaussian_block": (_c_i32, [_c_p, _c_i64, _c_i64, _c_i64, _c_i64, _c_p]),
    "rcqr_intermediates": (_c_i32, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "rcqr_q0_twice": (_c_i32, [_c_p, _c_p, _c_i64, _c_p, _c_p, _c_i64]),
    "rcqr_tune": (_c_i32, [_c_p, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64, _c_i32, ctypes.POINTER(ctypes.c_float)]),
    "rcqr_set_tuning": (_c_i32, [_c_p, _c_i32, _c_i32]),
    "rcqr_get_tuning": (_c_i32, [_c_p, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "rcqr_graph_create": (_c_i32, [_c_p, _c_i32, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64, ctypes.POINTER(_c_p)]),
    "rcqr_graph_launch": (_c_i32, [_c_p]),
    "rcqr_graph_destroy": (_c_i32, [_c_p]),
    "rcqr_batch_create": (_c_i32, [_c_i32, ctypes.POINTER(_c_p), _c_i32, ctypes.POINTER(_c_p), ctypes.POINTER(_c_i64),
                                   ctypes.POINTER(_c_p), ctypes.POINTER(_c_i64), ctypes.POINTER(_c_p), ctypes.POINTER(_c_i64),
                                   ctypes.POINTER(_c_p)]),
    "rcqr_batch_launch": (_c_i32, [_c_p]),
    "rcqr_factor_batch": (_c_i32, [_c_p, _c_i32, _c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i64, _c_p]),
    "rcqr_info_member": (_c_i32, [_c_p, _c_i32, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "rcqr_info_batch": (_c_i32, [_c_p, _c_i32, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "rcqr_batch_destroy": (_c_i32, [_c_p]),
    "rcqr_factor_ragged": (_c_i32, [_c_p, _c_i32, _c_p]),
    "rcqr_factor_static": (_c_i32, [_c_i64, _c_i64, _c_i64, _c_i64, _c_u64, _c_u32, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_i64, _c_p,
                                    _c_p]),
}


class _RaggedMember(ctypes.Structure):
    """rcqr_member_t of include/rcqr.h."""
    _fields_ = [("V", _c_p), ("Q", _c_p), ("R", _c_p), ("m", _c_i64), ("ldv", _c_i64), ("ldq", _c_i64), ("ldr", _c_i64),
                ("seed", _c_u64)]


# rcqr_member_t as one numpy record (the same 64-byte layout as _RaggedMember)
def _member_dtype():
    import numpy as np

    return np.dtype([("V", "<u8"), ("Q", "<u8"), ("R", "<u8"), ("m", "<i8"), ("ldv", "<i8"), ("ldq", "<i8"), ("ldr", "<i8"),
                     ("seed", "<u8")])


_MEMBER_DTYPE = _member_dtype()
assert _MEMBER_DTYPE.itemsize == ctypes.sizeof(_RaggedMember)


class RcqrError(RuntimeError):
    def __init__(self, status, what, column=0):
        self.status = int(status)
        self.column = int(column)
        msg = f"{what}: {status_string(status)} (status {status}"
        msg += f", column {column})" if column else ")"
        super().__init__(msg)


def declared_functions(header=HEADER_PATH):
    """Names of the functions include/rcqr.h declares."""
    with open(header) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    return sorted(set(re.findall(r"\b(rcqr_\w+)\s*\(", text)))


def lib():
    """The loaded librcqr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2309_05868_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status):
    return lib().rcqr_status_string(int(status)).decode()


def _check(status, what):
    if status != OK:
        raise RcqrError(status, what)


def workspace_bytes(m, n, s1, s2, flags=0):
    return int(lib().rcqr_workspace_bytes(m, n, s1, s2, flags))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_matrix(V, m, n, name):
    if not isinstance(V, torch.Tensor) or V.dtype != torch.float64 or not V.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    if V.dim() != 2 or tuple(V.shape) != (m, n) or V.stride(1) != 1 or V.stride(0) < n:
        raise ValueError(f"{name} must be a row-major {m} x {n} matrix with unit column stride")


class Plan:
    """A factorization plan for m x n inputs with CountSketch size s1, Gaussian size s2, seed
    (flags: FLAG_* bits, 0 = all FP64)."""

    def __init__(self, m, n, s1, s2, seed, device=None, stream=None, flags=0, batch=1):
        self.m, self.n, self.s1, self.s2, self.seed = int(m), int(n), int(s1), int(s2), int(seed)
        self.flags = int(flags)
        self.batch = int(batch)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = workspace_bytes(self.m, self.n, self.s1, self.s2, self.flags)
        if nbytes == 0 or self.batch < 1:
            raise RcqrError(E_UNSUPPORTED if 0 < n and n > MAX_N else E_INVALID, "rcqr_workspace_bytes")
        nbytes *= self.batch  # one workspace slice per batch member (factor_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        _check(lib().rcqr_plan(ctypes.byref(handle), self.m, self.n, self.s1, self.s2, self.seed, self.flags,
                               ctypes.c_void_p(self.workspace.data_ptr()), nbytes, _stream_ptr(self.stream)), "rcqr_plan")
        self._h = handle

    # -- lifecycle ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().rcqr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- factorizations ------------------------------------------------------------------
    def _outputs(self, V, Q, R):
        _check_matrix(V, self.m, self.n, "V")
        if Q is None:
            Q = torch.empty((self.m, self.n), dtype=torch.float64, device=V.device)
        if R is None:
            R = torch.empty((self.n, self.n), dtype=torch.float64, device=V.device)
        _check_matrix(Q, self.m, self.n, "Q")
        _check_matrix(R, self.n, self.n, "R")
        return Q, R

    def _call(self, name, V, Q, R, check):
        Q, R = self._outputs(V, Q, R)
        _check(getattr(lib(), name)(self._h, ctypes.c_void_p(V.data_ptr()), V.stride(0), ctypes.c_void_p(Q.data_ptr()),
                                    Q.stride(0), ctypes.c_void_p(R.data_ptr()), R.stride(0)), name)
        if check:
            self.raise_on_failure(name)
        return Q, R

    def factor(self, V, Q=None, R=None, check=True):
        """Algorithm 3 on V; returns (Q, R).  With check=True waits and raises on RANK/CHOL."""
        return self._call("rcqr_factor", V, Q, R, check)

    def cholqr2(self, V, Q=None, R=None, check=True):
        """Algorithm 4 (cholQR2) on V with this plan's workspace; returns (Q, R)."""
        return self._call("rcqr_cholqr2", V, Q, R, check)

    def scholqr3(self, V, Q=None, R=None, check=True):
        """Shifted CholeskyQR3 on V with this plan's workspace; returns (Q, R)."""
        return self._call("rcqr_scholqr3", V, Q, R, check)

    def info(self):
        st, col = _c_i32(), _c_i32()
        _check(lib().rcqr_info(self._h, ctypes.byref(st), ctypes.byref(col)), "rcqr_info")
        return st.value, col.value

    def raise_on_failure(self, what):
        st, col = self.info()
        if st != OK:
            raise RcqrError(st, what, col)

    def tune(self, V, reps=3):
        """Time the result-neutral launch choices on V and keep the fastest; returns
        (final_mode, grid_mult, ms per factorization).  Synchronises the plan's stream."""
        Q, R = self._outputs(V, None, None)
        best = ctypes.c_float()
        _check(lib().rcqr_tune(self._h, ctypes.c_void_p(V.data_ptr()), V.stride(0), ctypes.c_void_p(Q.data_ptr()), Q.stride(0),
                               ctypes.c_void_p(R.data_ptr()), R.stride(0), int(reps), ctypes.byref(best)), "rcqr_tune")
        mode, mult = self.tuning()
        return mode, mult, float(best.value)

    def tuning(self):
        mode, mult = _c_i32(), _c_i32()
        _check(lib().rcqr_get_tuning(self._h, ctypes.byref(mode), ctypes.byref(mult)), "rcqr_get_tuning")
        return mode.value, mult.value

    def set_tuning(self, final_mode, grid_mult):
        _check(lib().rcqr_set_tuning(self._h, int(final_mode), int(grid_mult)), "rcqr_set_tuning")

    def factor_batch(self, V, Q=None, R=None, seeds=None):
        """rcqr_factor_batch: V of shape (count, m, n), count <= the plan's batch; member b uses
        seeds[b] (a CUDA int64/uint64 tensor of count seeds) or, without seeds, the plan's seed + b.
        Returns (Q, R) of shapes (count, m, n) and (count, n, n)."""
        if V.dim() != 3 or V.shape[1:] != (self.m, self.n) or V.dtype != torch.float64 or not V.is_cuda:
            raise ValueError("V must be a CUDA float64 tensor of shape (count, m, n)")
        k = V.shape[0]
        if Q is None:
            Q = torch.empty_like(V)
        if R is None:
            R = torch.empty((k, self.n, self.n), dtype=torch.float64, device=V.device)
        for t, nm in ((V, "V"), (Q, "Q"), (R, "R")):
            if t.stride(2) != 1:
                raise ValueError(f"{nm} rows must be contiguous")
        sp = None
        if seeds is not None:
            if not seeds.is_cuda or seeds.dtype not in (torch.int64, torch.uint64) or seeds.numel() < k or not seeds.is_contiguous():
                raise ValueError("seeds must be a contiguous CUDA int64 tensor with one seed per member")
            sp = ctypes.c_void_p(seeds.data_ptr())
        _check(lib().rcqr_factor_batch(self._h, k, ctypes.c_void_p(V.data_ptr()), V.stride(1), V.stride(0),
                                       ctypes.c_void_p(Q.data_ptr()), Q.stride(1), Q.stride(0),
                                       ctypes.c_void_p(R.data_ptr()), R.stride(1), R.stride(0), sp), "rcqr_factor_batch")
        return Q, R

    def factor_ragged(self, Vs, Qs=None, Rs=None, seeds=None):
        """rcqr_factor_ragged: Algorithm 3 on matrices of the plan's n, s1, s2 and their own row
        counts (each at most the plan's m), in one set of launches.  Vs: list of CUDA float64
        row-major tensors; Qs / Rs: outputs (allocated when None, as views of one tensor each; Q
        may be V); seeds: one int per member (default: the plan's seed + b).  Returns (Qs, Rs);
        statuses via info_batch.  The member table is built as one array (a serving loop calls
        this once per batch)."""
        import numpy as np

        k = len(Vs)
        if k < 1 or k > self.batch:
            raise ValueError(f"need 1 .. {self.batch} members (the plan's batch)")
        n = self.n
        f64 = torch.float64
        for b, V in enumerate(Vs):  # one cheap test per member; the full check names the problem
            if not (isinstance(V, torch.Tensor) and V.dtype is f64 and V.is_cuda and V.dim() == 2 and V.shape[1] == n
                    and V.stride(1) == 1 and V.stride(0) >= n):
                _check_matrix(V, V.shape[0] if V.dim() == 2 else -1, n, f"V[{b}]")
        ms = [V.shape[0] for V in Vs]
        dev = Vs[0].device
        Qs = list(Qs) if Qs is not None else [None] * k
        Rs = list(Rs) if Rs is not None else [None] * k
        for b in range(k):  # caller-given outputs are checked; fresh ones are views of one tensor
            if Qs[b] is not None:
                _check_matrix(Qs[b], ms[b], n, f"Q[{b}]")
            if Rs[b] is not None:
                _check_matrix(Rs[b], n, n, f"R[{b}]")
        miss = [b for b in range(k) if Qs[b] is None]
        if miss:
            qall = torch.empty((sum(ms[b] for b in miss), n), dtype=f64, device=dev)
            for b, Q in zip(miss, torch.split(qall, [ms[b] for b in miss])):
                Qs[b] = Q
        miss = [b for b in range(k) if Rs[b] is None]
        if miss:
            for b, R in zip(miss, torch.empty((len(miss), n, n), dtype=f64, device=dev).unbind(0)):
                Rs[b] = R
        seeds = list(seeds) if seeds is not None else [self.seed + b for b in range(k)]
        table = np.array([(V.data_ptr(), Q.data_ptr(), R.data_ptr(), m, V.stride(0), Q.stride(0), R.stride(0),
                           int(sd) & 0xFFFFFFFFFFFFFFFF) for V, Q, R, m, sd in zip(Vs, Qs, Rs, ms, seeds)], dtype=_MEMBER_DTYPE)
        _check(lib().rcqr_factor_ragged(self._h, k, ctypes.c_void_p(table.ctypes.data)), "rcqr_factor_ragged")
        self._ragged_keep = (Vs, Qs, Rs)  # the buffers stay referenced until the next call
        return Qs, Rs

    def info_batch(self, count):
        """[(status, column)] of members 0 .. count-1, one device-to-host copy."""
        st, col = (_c_i32 * int(count))(), (_c_i32 * int(count))()
        _check(lib().rcqr_info_batch(self._h, int(count), st, col), "rcqr_info_batch")
        return [(st[i], col[i]) for i in range(int(count))]

    def info_member(self, b):
        st, col = _c_i32(), _c_i32()
        _check(lib().rcqr_info_member(self._h, int(b), ctypes.byref(st), ctypes.byref(col)), "rcqr_info_member")
        return st.value, col.value

    def graph(self, V, Q=None, R=None, method="rand_cholqr"):
        """Capture one factorization of V into (Q, R) as a HIP graph; returns a Graph whose
        launch() replays it on this plan's stream.  Needs a plan on a non-default stream."""
        Q, R = self._outputs(V, Q, R)
        h = ctypes.c_void_p()
        _check(lib().rcqr_graph_create(self._h, METHODS[method], ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                       ctypes.c_void_p(Q.data_ptr()), Q.stride(0), ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                       ctypes.byref(h)), "rcqr_graph_create")
        return Graph(self, h, V, Q, R)

    # -- timing ----------------------------------------------------------------------------
    def set_timing(self, steps=1):
        """Record per-phase HIP events for the next `steps` factor calls (0 turns it off)."""
        _check(lib().rcqr_set_timing(self._h, int(steps)), "rcqr_set_timing")

    def phase_times(self):
        """Mean per-phase milliseconds over the factor calls recorded since the last read."""
        arr = (ctypes.c_float * 16)()
        cnt = _c_i32()
        _check(lib().rcqr_phase_times(self._h, arr, 16, ctypes.byref(cnt)), "rcqr_phase_times")
        return {lib().rcqr_phase_name(i).decode(): float(arr[i]) for i in range(cnt.value)}

    # -- inspection --------------------------------------------------------------------------
    def sketch_hash(self, row0, count):
        b = torch.empty(count, dtype=torch.int32, device=self.device)
        g = torch.empty(count, dtype=torch.int8, device=self.device)
        _check(lib().rcqr_sketch_hash(self._h, row0, count, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(g.data_ptr())),
               "rcqr_sketch_hash")
        return b, g

    def gaussian_block(self, j0, nj, k0, nk):
        out = torch.empty((nj, nk), dtype=torch.float64, device=self.device)
        _check(lib().rcqr_gaussian_block(self._h, j0, nj, k0, nk, ctypes.c_void_p(out.data_ptr())), "rcqr_gaussian_block")
        return out

    def intermediates(self):
        f = lambda *s: torch.empty(s, dtype=torch.float64, device=self.device)  # noqa: E731
        out = {"W1": f(self.s1, self.n), "W": f(self.s2, self.n), "R0": f(self.n, self.n), "G": f(self.n, self.n),
               "R1": f(self.n, self.n)}
        ptr = {k: ctypes.c_void_p(v.data_ptr()) for k, v in out.items()}
        _check(lib().rcqr_intermediates(self._h, ptr["W1"], ptr["W"], ptr["R0"], ptr["G"], ptr["R1"]), "rcqr_intermediates")
        return out

    def q0_twice(self, V):
        _check_matrix(V, self.m, self.n, "V")
        a = torch.empty((self.m, self.n), dtype=torch.float64, device=V.device)
        b = torch.empty_like(a)
        _check(lib().rcqr_q0_twice(self._h, ctypes.c_void_p(V.data_ptr()), V.stride(0), ctypes.c_void_p(a.data_ptr()),
                                   ctypes.c_void_p(b.data_ptr()), self.n), "rcqr_q0_twice")
        return a, b


class Graph:
    """A captured factorization (rcqr_graph_*): keeps the plan and the tensors it reads and
    writes alive; launch() replays it, close() frees it (before the plan)."""

    def __init__(self, plan, handle, V, Q, R):
        self.plan, self._h, self.V, self.Q, self.R = plan, handle, V, Q, R

    def launch(self, check=False):
        _check(lib().rcqr_graph_launch(self._h), "rcqr_graph_launch")
        if check:
            self.plan.raise_on_failure("rcqr_graph_launch")
        return self.Q, self.R

    def close(self):
        if getattr(self, "_h", None):
            lib().rcqr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several factorizations launched together (rcqr_batch_*): each member captured as a HIP
    graph on its plan's stream, all launched concurrently, forked from and joined to plans[0]'s
    stream.  plans[i] factors Vs[i] into Qs[i], Rs[i]; each plan needs its own non-default
    stream."""

    def __init__(self, plans, Vs, Qs=None, Rs=None, method="rand_cholqr"):
        k = len(plans)
        if k < 1 or len(Vs) != k:
            raise ValueError("need one V per plan")
        Qs = list(Qs) if Qs is not None else [None] * k
        Rs = list(Rs) if Rs is not None else [None] * k
        outs = [p._outputs(V, Q, R) for p, V, Q, R in zip(plans, Vs, Qs, Rs)]
        self.plans, self.Vs = list(plans), list(Vs)
        self.Qs, self.Rs = [o[0] for o in outs], [o[1] for o in outs]
        P = (_c_p * k)(*[p._h for p in plans])
        ptr = lambda ts: (_c_p * k)(*[t.data_ptr() for t in ts])  # noqa: E731
        ld = lambda ts: (_c_i64 * k)(*[t.stride(0) for t in ts])  # noqa: E731
        h = ctypes.c_void_p()
        _check(lib().rcqr_batch_create(k, P, METHODS[method], ptr(self.Vs), ld(self.Vs), ptr(self.Qs), ld(self.Qs),
                                       ptr(self.Rs), ld(self.Rs), ctypes.byref(h)), "rcqr_batch_create")
        self._h = h

    def launch(self):
        _check(lib().rcqr_batch_launch(self._h), "rcqr_batch_launch")
        return self.Qs, self.Rs

    def close(self):
        if getattr(self, "_h", None):
            lib().rcqr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_static(V, Q, R, s1, s2, seed, info=None, flags=0, stream=None):
    """rcqr_factor_static: Algorithm 3 on V into the caller's Q and R with the library's static
    per-GPU workspace (no plan, no device allocation by the library).  info: None or a CUDA int32
    tensor of two entries that receives (status, failing column) in stream order.  Enqueued on
    `stream` (default: the current stream) and not waited for."""
    m, n = V.shape
    _check_matrix(V, m, n, "V")
    _check_matrix(Q, m, n, "Q")
    _check_matrix(R, n, n, "R")
    ip = None
    if info is not None:
        if not info.is_cuda or info.dtype != torch.int32 or info.numel() < 2 or not info.is_contiguous():
            raise ValueError("info must be a contiguous CUDA int32 tensor of two entries")
        ip = ctypes.c_void_p(info.data_ptr())
    _check(lib().rcqr_factor_static(m, n, int(s1), int(s2), int(seed), int(flags), ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                    ctypes.c_void_p(Q.data_ptr()), Q.stride(0), ctypes.c_void_p(R.data_ptr()), R.stride(0), ip,
                                    _stream_ptr(stream)), "rcqr_factor_static")
    return Q, R


def rand_cholqr(V, s1, s2, seed, check=True, flags=0):
    """One-shot Algorithm 3: returns (Q, R) for the CUDA float64 matrix V."""
    m, n = V.shape
    with Plan(m, n, s1, s2, seed, device=V.device, flags=flags) as p:
        Q, R = p.factor(V, check=check)
        torch.cuda.current_stream(V.device).synchronize()
        return Q, R


def cholqr2(V, check=True):
    """One-shot Algorithm 4 (cholQR2) on the GPU; returns (Q, R)."""
    m, n = V.shape
    with Plan(m, n, max(n, 16), n, 0, device=V.device) as p:
        Q, R = p.cholqr2(V, check=check)
        torch.cuda.current_stream(V.device).synchronize()
        return Q, R


def scholqr3(V, check=True):
    """One-shot shifted CholeskyQR3 on the GPU; returns (Q, R)."""
    m, n = V.shape
    with Plan(m, n, max(n, 16), n, 0, device=V.device) as p:
        Q, R = p.scholqr3(V, check=check)
        torch.cuda.current_stream(V.device).synchronize()
        return Q, R
