"""Python binding of libadr.so: the MI355X ETD2RKds hot path.

A thin ctypes layer over the C ABI declared in ``include/adr.h``: every
function here marshals arguments and calls the entry point of the same name;
all arithmetic of the method runs in the library's HIP kernels.  PyTorch is
only used to own device memory and to name the current HIP stream.

``torch`` is imported before the library is loaded so that both use one HIP
runtime.  If ``libadr.so`` has not been built the import fails loudly; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (load torch's HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadr.so")

ADR_OK, ADR_EINVAL, ADR_ENOMEM, ADR_EDEVICE, ADR_ENOTSUP, ADR_ENONFINITE = 0, -1, -2, -3, -4, -5
ADR_BC_NEUMANN = 0
ADR_ETD2RKDS, ADR_LAWSON2B = 0, 1
ADR_F64, ADR_F32, ADR_BF16X3, ADR_BF16X2 = 0, 1, 2, 3
ADR_SCHNAKENBERG, ADR_FHN, ADR_BRUSSELATOR, ADR_ZERO, ADR_DIB = 0, 1, 2, 3, 4
ADR_MAX_PARAMS = 12
ADR_PHI_NOALLOC_MAX_N = 512
ADR_BATCH_AUTOTUNE, ADR_BATCH_GRAPH, ADR_BATCH_PREPARED = 1, 2, 4


def ADR_BATCH_TILE(cfg: int) -> int:
    """Flag forcing tile configuration cfg (0..3) for the FP64 mode-product phases."""
    return (int(cfg) + 1) << 8

MODEL_IDS = {"schnakenberg": ADR_SCHNAKENBERG, "fhn": ADR_FHN,
             "brusselator": ADR_BRUSSELATOR, "zero": ADR_ZERO, "dib": ADR_DIB}
SCHEME_IDS = {"etd2rkds": ADR_ETD2RKDS, "lawson2b": ADR_LAWSON2B}
PRECISION_IDS = {"f64": ADR_F64, "f32": ADR_F32, "bf16x3": ADR_BF16X3, "bf16x2": ADR_BF16X2}

_dp = ctypes.POINTER(ctypes.c_double)


class AdrProblem(ctypes.Structure):
    """Mirror of ``adr_problem`` in include/adr.h."""

    _fields_ = [
        ("d", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("model", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("params", ctypes.c_double * 12),
        ("tau", ctypes.c_double),
        ("phi", ((ctypes.c_void_p * 3) * 3) * 2),
        ("band", (ctypes.c_void_p * 3) * 2),
        ("dense", (ctypes.c_void_p * 3) * 2),
    ]


class AdrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {adr_strerror(status)} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_2307_10684_amd/build.py` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_size, c_void = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "adr_strerror": (ctypes.c_char_p, [c_int]),
        "adr_version": (c_int, []),
        "adr_build_1d_ops": (c_int, [c_int, c_double, c_double, c_double, c_double, c_int, c_void, c_void]),
        "adr_precompute_phi": (c_int, [c_int, c_void, c_double, c_void, c_void, c_void, c_void]),
        "adr_precompute_phi_noalloc": (c_int, [c_int, c_void, c_double, c_void, c_void, c_void, c_void]),
        "adr_precompute_phi_batch": (c_int, [c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_void),
                                             ctypes.POINTER(c_double), ctypes.POINTER(c_void),
                                             ctypes.POINTER(c_void), ctypes.POINTER(c_void), c_void]),
        "adr_workspace_bytes": (c_size, [ctypes.POINTER(AdrProblem)]),
        "adr_step": (c_int, [ctypes.POINTER(AdrProblem), c_void, c_void, c_void, c_size, c_void]),
        "adr_solve": (c_int, [ctypes.POINTER(AdrProblem), c_void, c_void, c_int, c_void, c_size, c_void]),
        "adr_mode_product": (c_int, [c_int, ctypes.POINTER(ctypes.c_int32), c_int, c_void, c_void, c_void,
                                     c_double, c_double, c_void, c_void]),
        "adr_tucker_workspace_bytes": (c_size, [c_int, ctypes.POINTER(ctypes.c_int32)]),
        "adr_tucker": (c_int, [c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_void), c_void, c_void,
                               c_double, c_double, c_void, c_void, c_size, c_void]),
        "adr_device_copy": (c_int, [c_void, c_void, c_size, c_void]),
        "adr_timing_enable": (c_int, [c_int]),
        "adr_timing_read": (c_int, [c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
        "adr_indicators_workspace_bytes": (c_size, [c_int, ctypes.POINTER(ctypes.c_int32)]),
        "adr_indicators": (c_int, [c_int, ctypes.POINTER(ctypes.c_int32), c_void, c_void, c_void, c_void,
                                   c_void, c_void, c_size, c_void]),
        "adr_monitor_workspace_bytes": (c_size, [ctypes.POINTER(AdrProblem)]),
        "adr_solve_monitored": (c_int, [ctypes.POINTER(AdrProblem), c_void, c_void, c_int, c_int, c_void,
                                        c_void, c_size, c_void, c_size, c_void]),
        "adr_batch_create": (c_int, [c_int, ctypes.POINTER(AdrProblem), ctypes.POINTER(c_void),
                                     ctypes.POINTER(c_void), ctypes.POINTER(c_void),
                                     ctypes.POINTER(c_size), c_int, c_void, ctypes.POINTER(c_void)]),
        "adr_batch_run": (c_int, [c_void, c_int, c_void]),
        "adr_batch_info": (c_int, [c_void, ctypes.POINTER(c_int), c_int, ctypes.POINTER(c_int)]),
        "adr_batch_destroy": (c_int, [c_void]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("adr_strerror", "adr_version", "adr_build_1d_ops", "adr_precompute_phi",
            "adr_precompute_phi_noalloc", "adr_precompute_phi_batch",
            "adr_workspace_bytes", "adr_step", "adr_solve", "adr_mode_product",
            "adr_tucker_workspace_bytes", "adr_tucker", "adr_device_copy",
            "adr_timing_enable", "adr_timing_read", "adr_indicators_workspace_bytes",
            "adr_indicators", "adr_monitor_workspace_bytes", "adr_solve_monitored",
            "adr_batch_create", "adr_batch_run", "adr_batch_info", "adr_batch_destroy")


def _check(status: int, where: str):
    if status != ADR_OK:
        raise AdrError(status, where)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dims(n: Sequence[int]):
    arr = (ctypes.c_int32 * 3)(*(list(n) + [1] * (3 - len(n))))
    return arr


def _f64_cuda(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")


# ----------------------------------------------------------------------------- ABI wrappers

def adr_strerror(status: int) -> str:
    return _lib.adr_strerror(status).decode()


def adr_version() -> int:
    return _lib.adr_version()


def adr_build_1d_ops(n: int, a: float, b: float, diff: float, vel: float, bc: int = ADR_BC_NEUMANN):
    """Host call: returns (A (n x n, numpy, column-major semantics), band (3, n))."""
    A = np.zeros((n, n), dtype=np.float64, order="F")
    band = np.zeros(3 * n, dtype=np.float64)
    _check(_lib.adr_build_1d_ops(n, a, b, diff, vel, bc, A.ctypes.data, band.ctypes.data),
           "adr_build_1d_ops")
    return A, band.reshape(3, n)


def adr_precompute_phi(A_dev: torch.Tensor, tau: float, E=None, P1=None, P2=None, stream=None,
                       want=(True, True, True)):
    """E, phi_1, phi_2 of tau*A on the device.  A_dev is an (n, n) float64 CUDA tensor
    holding the column-major matrix (i.e. the transpose in torch's row-major view
    is never taken: pass ``torch.from_numpy(A.ravel(order='F'))``-style data)."""
    n = int(round(math.sqrt(A_dev.numel())))
    _f64_cuda(A_dev, "A_dev")
    outs = []
    for t, w in zip((E, P1, P2), want):
        if t is None and w:
            t = torch.empty(n * n, dtype=torch.float64, device=A_dev.device)
        outs.append(t)
    _check(_lib.adr_precompute_phi(n, _ptr(A_dev), float(tau), _ptr(outs[0]), _ptr(outs[1]),
                                   _ptr(outs[2]), _stream(stream)), "adr_precompute_phi")
    return tuple(outs)


def adr_precompute_phi_noalloc(A_dev: torch.Tensor, tau: float, E=None, P1=None, P2=None,
                               stream=None, want=(True, True, True)):
    """adr_precompute_phi in the library's fixed per-GPU work area (no device
    allocation inside the call; n <= ADR_PHI_NOALLOC_MAX_N).  Outputs that are
    not given are allocated here, before the call."""
    n = int(round(math.sqrt(A_dev.numel())))
    _f64_cuda(A_dev, "A_dev")
    outs = []
    for t, w in zip((E, P1, P2), want):
        if t is None and w:
            t = torch.empty(n * n, dtype=torch.float64, device=A_dev.device)
        outs.append(t)
    _check(_lib.adr_precompute_phi_noalloc(n, _ptr(A_dev), float(tau), _ptr(outs[0]),
                                           _ptr(outs[1]), _ptr(outs[2]), _stream(stream)),
           "adr_precompute_phi_noalloc")
    return tuple(outs)


def adr_precompute_phi_batch(As, taus, stream=None):
    """E, phi_1, phi_2 of tau_i * A_i for several device matrices (each an (n_i * n_i,)
    float64 CUDA tensor, column-major) in one call with two synchronisations.
    Returns a list of (E, P1, P2) tensors."""
    count = len(As)
    if len(taus) != count or count == 0:
        raise ValueError("As and taus must be non-empty and of the same length")
    ns, outs = [], []
    for A in As:
        _f64_cuda(A, "A_dev")
        n = int(round(math.sqrt(A.numel())))
        ns.append(n)
        outs.append(tuple(torch.empty(n * n, dtype=torch.float64, device=A.device) for _ in range(3)))
    n_arr = (ctypes.c_int32 * count)(*ns)
    a_arr = (ctypes.c_void_p * count)(*[_ptr(A) for A in As])
    t_arr = (ctypes.c_double * count)(*[float(t) for t in taus])
    e_arr, p1_arr, p2_arr = ((ctypes.c_void_p * count)(*[_ptr(o[j]) for o in outs]) for j in range(3))
    _check(_lib.adr_precompute_phi_batch(count, n_arr, a_arr, t_arr, e_arr, p1_arr, p2_arr,
                                         _stream(stream)), "adr_precompute_phi_batch")
    return outs


def adr_workspace_bytes(problem: AdrProblem) -> int:
    return int(_lib.adr_workspace_bytes(ctypes.byref(problem)))


def adr_step(problem: AdrProblem, U, V, work, stream=None):
    _check(_lib.adr_step(ctypes.byref(problem), _ptr(U), _ptr(V), _ptr(work),
                         work.numel() * work.element_size(), _stream(stream)), "adr_step")


def adr_solve(problem: AdrProblem, U, V, nsteps: int, work, stream=None):
    _check(_lib.adr_solve(ctypes.byref(problem), _ptr(U), _ptr(V), int(nsteps), _ptr(work),
                          work.numel() * work.element_size(), _stream(stream)), "adr_solve")


def adr_mode_product(n: Sequence[int], mu: int, M, W, out, alpha=1.0, beta=0.0, Y=None, stream=None):
    _check(_lib.adr_mode_product(len(n), _dims(n), mu, _ptr(M), _ptr(W), _ptr(out), float(alpha),
                                 float(beta), _ptr(Y), _stream(stream)), "adr_mode_product")


def adr_tucker_workspace_bytes(n: Sequence[int]) -> int:
    return int(_lib.adr_tucker_workspace_bytes(len(n), _dims(n)))


def adr_tucker(n: Sequence[int], Ms, W, out, alpha=1.0, beta=0.0, Y=None, work=None, stream=None):
    arr = (ctypes.c_void_p * len(n))(*[_ptr(M) for M in Ms])
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(_lib.adr_tucker(len(n), _dims(n), arr, _ptr(W), _ptr(out), float(alpha), float(beta),
                           _ptr(Y), _ptr(work), wb, _stream(stream)), "adr_tucker")


def adr_device_copy(src, dst, count: int, stream=None):
    _check(_lib.adr_device_copy(_ptr(src), _ptr(dst), int(count), _stream(stream)), "adr_device_copy")


def adr_timing_enable(capacity: int):
    _check(_lib.adr_timing_enable(int(capacity)), "adr_timing_enable")


def adr_timing_read(kind: int):
    launches = ctypes.c_int(0)
    total = ctypes.c_double(0.0)
    _check(_lib.adr_timing_read(int(kind), ctypes.byref(launches), ctypes.byref(total)),
           "adr_timing_read")
    return launches.value, total.value


def adr_indicators_workspace_bytes(n: Sequence[int]) -> int:
    return int(_lib.adr_indicators_workspace_bytes(len(n), _dims(n)))


def adr_indicators(n: Sequence[int], U, V, Uprev=None, Vprev=None, rec=None, work=None,
                   stream=None):
    """The five indicators of (U, V) (and the increment from (Uprev, Vprev)) into the
    device tensor ``rec`` (5 doubles, allocated if not given); returns ``rec``."""
    dev = U.device
    if rec is None:
        rec = torch.empty(5, dtype=torch.float64, device=dev)
    if work is None:
        work = torch.empty((adr_indicators_workspace_bytes(n) + 7) // 8, dtype=torch.float64,
                           device=dev)
    _check(_lib.adr_indicators(len(n), _dims(n), _ptr(U), _ptr(V), _ptr(Uprev), _ptr(Vprev),
                               _ptr(rec), _ptr(work), work.numel() * work.element_size(),
                               _stream(stream)), "adr_indicators")
    return rec


def adr_monitor_workspace_bytes(problem: AdrProblem) -> int:
    return int(_lib.adr_monitor_workspace_bytes(ctypes.byref(problem)))


def adr_solve_monitored(problem: AdrProblem, U, V, nsteps: int, every: int, rec, work, mwork,
                        stream=None) -> int:
    """Returns ADR_OK or ADR_ENONFINITE (a record counted non-finite values);
    raises on other errors."""
    st = _lib.adr_solve_monitored(ctypes.byref(problem), _ptr(U), _ptr(V), int(nsteps),
                                  int(every), _ptr(rec), _ptr(work),
                                  work.numel() * work.element_size(), _ptr(mwork),
                                  mwork.numel() * mwork.element_size(), _stream(stream))
    if st not in (ADR_OK, ADR_ENONFINITE):
        raise AdrError(st, "adr_solve_monitored")
    return st


def adr_batch_create(problems: Sequence[AdrProblem], U, V, works, flags: int = 0, stream=None) -> int:
    """Build a grouped plan over ``len(problems)`` problems; returns the plan handle."""
    count = len(problems)
    if not (len(U) == len(V) == len(works) == count):
        raise ValueError("problems, U, V and works must have the same length")
    probs = (AdrProblem * count)(*problems)
    u = (ctypes.c_void_p * count)(*[_ptr(t) for t in U])
    v = (ctypes.c_void_p * count)(*[_ptr(t) for t in V])
    w = (ctypes.c_void_p * count)(*[_ptr(t) for t in works])
    wb = (ctypes.c_size_t * count)(*[t.numel() * t.element_size() for t in works])
    plan = ctypes.c_void_p(None)
    _check(_lib.adr_batch_create(count, probs, u, v, w, wb, int(flags), _stream(stream),
                                 ctypes.byref(plan)), "adr_batch_create")
    return plan.value


def adr_batch_run(plan: int, nsteps: int, stream=None):
    _check(_lib.adr_batch_run(plan, int(nsteps), _stream(stream)), "adr_batch_run")


def adr_batch_info(plan: int, max_phases: int = 3):
    cfg = (ctypes.c_int * max(max_phases, 1))()
    graph = ctypes.c_int(0)
    _check(_lib.adr_batch_info(plan, cfg, int(max_phases), ctypes.byref(graph)), "adr_batch_info")
    return list(cfg)[:max_phases], bool(graph.value)


def adr_batch_destroy(plan: int):
    _check(_lib.adr_batch_destroy(plan), "adr_batch_destroy")


def workspace_bytes_for(n: Sequence[int], precision: str = "f64", scheme: str = "etd2rkds") -> int:
    """adr_workspace_bytes for a grid, before any device buffer exists (the size
    depends only on the grid, scheme and precision; the pointers are placeholders
    that the call checks for presence only)."""
    p = AdrProblem()
    p.d = len(n)
    for mu in range(3):
        p.n[mu] = int(n[mu]) if mu < p.d else 1
    p.model = ADR_ZERO
    p.scheme = SCHEME_IDS[scheme]
    p.precision = PRECISION_IDS[precision]
    p.tau = 1.0
    for c in range(2):
        for mu in range(p.d):
            for j in range(3):
                p.phi[c][j][mu] = 256
            p.band[c][mu] = 256
    nbytes = adr_workspace_bytes(p)
    if nbytes == 0:
        raise AdrError(ADR_EINVAL, "adr_workspace_bytes")
    return nbytes


# ----------------------------------------------------------------------------- problem setup

def to_device_f64(x: np.ndarray, device="cuda") -> torch.Tensor:
    """Upload a numpy array in its first-index-fastest (Fortran) element order."""
    flat = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel(order="F"))
    return torch.from_numpy(flat).to(device)


def from_device(t: torch.Tensor, shape) -> np.ndarray:
    return np.asfortranarray(t.detach().cpu().numpy().reshape(tuple(shape), order="F"))


class Solver:
    """Sets up one workload on the device: 1D operators, their matrix functions,
    the problem record and the workspace; then steps the state in place.

    ``workload`` is any object with the fields of ``synth.Workload`` (n,
    domain, diff, vel_u, vel_v, model, params, tau).  ``phis`` may supply the
    small matrices from elsewhere as ``phis[c][j][mu]`` numpy arrays (j = 0 exp,
    1 phi_1, 2 phi_2); by default they are computed on the device with
    adr_precompute_phi.
    """

    def __init__(self, workload, scheme: str = "etd2rkds", precision: str = "f64",
                 device: str = "cuda", phis=None, use_band: bool = True, stream=None):
        w = workload
        self.workload = w
        self.shape = tuple(int(x) for x in w.n)
        self.d = len(self.shape)
        self.N = int(np.prod(self.shape))
        self.device = device
        self.stream = stream
        self.A_host = [[None] * self.d for _ in range(2)]
        self.keep = []  # device buffers referenced by the problem record
        self.phi_matrices = 0   # distinct matrices whose functions were computed here
        p = AdrProblem()
        p.d = self.d
        for mu in range(3):
            p.n[mu] = self.shape[mu] if mu < self.d else 1
        p.model = MODEL_IDS[w.model]
        p.scheme = SCHEME_IDS[scheme]
        p.precision = PRECISION_IDS[precision]
        p.flags = 0
        for i, v in enumerate(w.params):
            p.params[i] = float(v)
        p.tau = float(w.tau)
        # the 1D operators; directions (and components) with the same size, domain,
        # diffusion and velocity share one device copy and one set of matrix functions
        distinct = {}
        slot = {}
        for c in range(2):
            vel = w.vel_u if c == 0 else w.vel_v
            for mu in range(self.d):
                a, b = w.domain[mu]
                key = (self.shape[mu], float(a), float(b), float(w.diff[c]), float(vel[mu]))
                if key not in distinct:
                    A, band = adr_build_1d_ops(self.shape[mu], a, b, w.diff[c], vel[mu])
                    A_dev = to_device_f64(A, device)
                    band_dev = torch.from_numpy(np.ascontiguousarray(band.ravel())).to(device)
                    self.keep += [A_dev, band_dev]
                    distinct[key] = (A, A_dev, band_dev)
                slot[(c, mu)] = key
                A, A_dev, band_dev = distinct[key]
                self.A_host[c][mu] = A
                p.dense[c][mu] = A_dev.data_ptr()
                if use_band:
                    p.band[c][mu] = band_dev.data_ptr()
        if phis is None:
            keys = list(distinct)
            funcs = adr_precompute_phi_batch([distinct[k][1] for k in keys], [w.tau] * len(keys),
                                             stream=stream)
            by_key = dict(zip(keys, funcs))
            self.phi_matrices = len(keys)
        for c in range(2):
            for mu in range(self.d):
                if phis is None:
                    E, P1, P2 = by_key[slot[(c, mu)]]
                else:
                    E, P1, P2 = (to_device_f64(phis[c][j][mu], device) for j in range(3))
                self.keep += [E, P1, P2]
                for j, t in enumerate((E, P1, P2)):
                    p.phi[c][j][mu] = t.data_ptr()
        self.problem = p
        nbytes = adr_workspace_bytes(p)
        if nbytes == 0:
            raise AdrError(ADR_EINVAL, "adr_workspace_bytes")
        self.work = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)

    def phi_host(self, c: int, j: int, mu: int) -> np.ndarray:
        """Download one small matrix (column-major n x n) for inspection."""
        n = self.shape[mu]
        t = torch.empty(n * n, dtype=torch.float64, device=self.device)
        ptr = self.problem.phi[c][j][mu]
        adr_device_copy(ptr, t, n * n, self.stream)
        torch.cuda.synchronize()
        return from_device(t, (n, n))

    def upload(self, U: np.ndarray, V: np.ndarray):
        return to_device_f64(U, self.device), to_device_f64(V, self.device)

    def download(self, U_dev, V_dev):
        return from_device(U_dev, self.shape), from_device(V_dev, self.shape)

    def step(self, U_dev, V_dev):
        adr_step(self.problem, U_dev, V_dev, self.work, self.stream)

    def solve(self, U_dev, V_dev, nsteps: int):
        adr_solve(self.problem, U_dev, V_dev, nsteps, self.work, self.stream)

    def solve_monitored(self, U_dev, V_dev, nsteps: int, every: int = 1):
        """Solve and record the indicators every `every` steps.  Returns
        (records as a (nsteps // every, 5) numpy array: <U>, <V>, ||dU||_F,
        ||dV||_F, non-finite count; status ADR_OK or ADR_ENONFINITE)."""
        k = max(nsteps // every, 1)
        rec = torch.zeros(5 * k, dtype=torch.float64, device=self.device)
        if getattr(self, "mwork", None) is None:
            nb = adr_monitor_workspace_bytes(self.problem)
            self.mwork = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        st = adr_solve_monitored(self.problem, U_dev, V_dev, nsteps, every, rec, self.work,
                                 self.mwork, self.stream)
        torch.cuda.synchronize()
        return rec.cpu().numpy().reshape(k, 5)[: nsteps // every], st


class Batch:
    """A grouped plan over several workloads (``Solver`` objects hold each
    problem's operators, matrix functions and workspace; ``states`` their
    device tensors).  ``run`` advances every problem by ``nsteps`` steps in
    grouped launches."""

    def __init__(self, solvers: Sequence[Solver], states, flags: int = 0, stream=None):
        self.solvers = list(solvers)
        self.states = list(states)
        self.stream = stream
        self.plan = adr_batch_create([s.problem for s in self.solvers],
                                     [u for u, _ in self.states], [v for _, v in self.states],
                                     [s.work for s in self.solvers], flags, stream)

    def run(self, nsteps: int):
        adr_batch_run(self.plan, nsteps, self.stream)

    def info(self, max_phases: int = 3):
        return adr_batch_info(self.plan, max_phases)

    def close(self):
        if self.plan:
            adr_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = [n for n in dir() if n.startswith(("adr_", "ADR_"))] + ["ADR_BATCH_TILE"] + [
    "AdrProblem", "AdrError", "Solver", "Batch", "to_device_f64", "from_device", "EXPORTED",
    "LIB_PATH"]
