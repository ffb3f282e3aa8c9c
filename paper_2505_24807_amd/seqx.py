"""Thin Python binding of libseqx (include/seqx.h): argument marshalling only.

Every step of the computation runs inside the HIP library; this module
converts NumPy arrays / torch device tensors to plain pointers and status
codes to exceptions.  It never falls back to a CPU path: when the library is
missing or no GPU is usable, calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import traceback
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseqx.so")

CIS, TDHF = 0, 1
FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
GUESS_GAP, GUESS_LEARNED, GUESS_USER, GUESS_GAP_PSPACE = 0, 1, 2, 3
MLP_NFEAT, MLP_NWEIGHTS, MLP_NPARAMS = 12, 18305, 18329
NPARAM = 11
HARTREE_EV = 27.211386245988

STATUS = {0: "OK", 1: "E_ARG", 2: "E_ELEMENT", 3: "E_OPEN_SHELL", 4: "E_GEOMETRY", 5: "E_NOMEM",
          6: "E_DEVICE", 7: "E_SCF_NOCONV", 8: "E_DAV_NOCONV", 9: "E_UNSTABLE", 10: "E_BUFSIZE", 11: "E_STATE"}


class SeqxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class ScfOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("ndiis", C.c_int32), ("integrals_only", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("theory", C.c_int32), ("nroots", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("max_subspace", C.c_int32), ("mem_budget_bytes", C.c_size_t), ("precision", C.c_int32),
                ("guess", C.c_int32), ("n_user_guess", C.c_int32), ("user_guess", C.POINTER(C.c_double)),
                ("batched", C.c_int32), ("pspace", C.c_int32), ("root_batch", C.c_int32), ("nguard", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("seed", C.c_uint64),
                ("init", C.c_int32)]


class TrainLog(C.Structure):
    _fields_ = [("n_epochs", C.c_int32), ("seconds", C.c_double), ("loss", C.c_double * 256)]


class Stats(C.Structure):
    _fields_ = [("scf_iterations", C.c_int32), ("dav_iterations", C.c_int32), ("n_sigma", C.c_int64),
                ("commutator", C.c_double), ("t_integrals_s", C.c_double), ("t_scf_s", C.c_double),
                ("t_davidson_s", C.c_double), ("t_sigma_s", C.c_double), ("time_to_roots_s", C.c_double * 64),
                ("n_history", C.c_int32), ("phase_ms", C.c_double * 5), ("phase_launches", C.c_int64 * 5),
                ("phase_flops", C.c_double * 5), ("phase_bytes", C.c_double * 5), ("dav_phase_ms", C.c_double * 8),
                ("n_sigma_fp64", C.c_int64), ("refine_iteration", C.c_int32), ("t_autotune_s", C.c_double),
                ("batched_graph", C.c_int32), ("tile_variant", C.c_int32 * 5), ("batched_sigma_flops", C.c_double),
                ("max_subspace_used", C.c_int32), ("subspace_cap", C.c_int32), ("n_collapses", C.c_int32),
                ("fp32_iteration", C.c_int32), ("n_sigma_bf16x3", C.c_int64)]

    DAV_PHASES = ["sigma", "projection", "subspace eig", "ritz+residual", "check", "precond", "collapse", "ortho"]

    PHASES = ["C_occ V", "(C_occ V) C_virt^T", "G(R)", "G C_virt", "C_occ^T (G C_virt) + de V"]


_lib = None

# device allocator callbacks of seqx_set_allocator: alloc(bytes, user) -> ptr, release(ptr, user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

MNDO, AM1, PM3, PARAMS_FILE = 0, 1, 2, 3

_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_I = C.POINTER(C.c_int32)


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libseqx.so from the package directory; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libseqx.so not found at {path}; build it with `python -m paper_2505_24807_amd.build`")
    # A process holds one HIP runtime.  PyTorch ships its own copy under the
    # same soname: when PyTorch is installed it is loaded first, so that this
    # library binds to that runtime and PyTorch's streams and device memory are
    # valid here (a library loaded first would leave PyTorch without a GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    sig = {
        "seqx_abi_version": (C.c_int, []),
        "seqx_validate": (C.c_int, [C.c_int32, _I, _I, _D, C.c_char_p, C.c_size_t]),
        "seqx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
        "seqx_destroy": (None, [C.c_void_p]),
        "seqx_last_error": (C.c_char_p, [C.c_void_p]),
        "seqx_set_params": (C.c_int, [C.c_void_p, C.c_int32, _I, _D]),
        "seqx_load_params": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p]),
        "seqx_set_allocator": (C.c_int, [C.c_void_p, ALLOC_FN, RELEASE_FN, C.c_void_p]),
        "seqx_prepare": (C.c_int, [C.c_void_p, C.c_int32, _I, _I, _D, C.POINTER(ScfOpts), C.POINTER(C.c_void_p)]),
        "seqx_job_free": (None, [C.c_void_p]),
        "seqx_dims": (C.c_int, [C.c_void_p, C.c_int32, _I, _I, _I]),
        "seqx_scf_results": (C.c_int, [C.c_void_p, C.c_int32, _D, _D, _D]),
        "seqx_core_hamiltonian": (C.c_int, [C.c_void_p, C.c_int32, _D]),
        "seqx_integrals": (C.c_int, [C.c_void_p, C.c_int32, _D, C.c_size_t, C.POINTER(C.c_size_t)]),
        "seqx_sigma": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _D, _D, _D, C.c_int32]),
        "seqx_sigma_device": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_int32]),
        "seqx_sigma_device_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_int32]),
        "seqx_solve": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts)]),
        "seqx_param_gradient": (C.c_int, [C.c_void_p, C.c_int32, _D, C.c_size_t, _I]),
        "seqx_spectrum": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, _D]),
        "seqx_broaden": (C.c_int, [C.c_void_p, C.c_int32, _D, _D, C.c_double, C.c_double, C.c_double, C.c_int32,
                                   _D]),
        "seqx_results": (C.c_int, [C.c_void_p, C.c_int32, _D, _D, _D, _D, _D]),
        "seqx_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
        "seqx_history": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _I, _D, _D]),
        "seqx_mlp_set_params": (C.c_int, [C.c_void_p, _F, C.c_size_t]),
        "seqx_mlp_get_params": (C.c_int, [C.c_void_p, _F, C.c_size_t, C.POINTER(C.c_size_t)]),
        "seqx_mlp_save": (C.c_int, [C.c_void_p, C.c_char_p]),
        "seqx_mlp_load": (C.c_int, [C.c_void_p, C.c_char_p]),
        "seqx_mlp_train": (C.c_int, [C.c_void_p, C.POINTER(TrainOpts), C.POINTER(TrainLog)]),
        "seqx_features": (C.c_int, [C.c_void_p, C.c_int32, _F, C.c_size_t]),
        "seqx_mlp_scores": (C.c_int, [C.c_void_p, C.c_int32, _F, C.c_size_t]),
        "seqx_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_int64, _F, _F, C.c_int32, C.POINTER(C.c_int64),
                                         C.POINTER(C.c_double), _F]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _fptr(a):
    return None if a is None else a.ctypes.data_as(_F)


def _iptr(a):
    return None if a is None else a.ctypes.data_as(_I)


def validate(natoms, Z, xyz):
    """Host-only input check; returns (status, message)."""
    lib = load_library()
    natoms = np.ascontiguousarray(natoms, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.int32)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    buf = C.create_string_buffer(512)
    s = lib.seqx_validate(len(natoms), _iptr(natoms), _iptr(Z), _dptr(xyz), buf, 512)
    return s, buf.value.decode()


@dataclass
class Results:
    omega_eV: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    f: np.ndarray
    mu: np.ndarray


class Context:
    """One GPU and one stream.  `stream`: a hipStream_t as int (torch's cuda_stream) or None."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.lib = load_library()
        self._callbacks = []
        self._jobs = weakref.WeakSet()
        self._exit_hook = False
        h = C.c_void_p()
        s = self.lib.seqx_create(device, C.c_void_p(stream) if stream else None, C.byref(h))
        if s != 0:
            raise SeqxError(s, self.lib.seqx_last_error(None).decode())
        self.h = h

    def _check(self, s):
        if s != 0:
            raise SeqxError(s, self.lib.seqx_last_error(self.h).decode())

    def set_params(self, Zs, values):
        Zs = np.ascontiguousarray(Zs, dtype=np.int32)
        values = np.ascontiguousarray(values, dtype=np.float64).reshape(len(Zs), NPARAM)
        self._check(self.lib.seqx_set_params(self.h, len(Zs), _iptr(Zs), _dptr(values)))

    def load_params(self, path: str, method: int = PARAMS_FILE):
        """seqx_load_params: a JSON parameter file (or a named method, which is not bundled)."""
        self._check(self.lib.seqx_load_params(self.h, method, path.encode() if path is not None else None))

    def set_allocator(self, alloc, release):
        """seqx_set_allocator with Python callables alloc(nbytes) -> device pointer (int) and
        release(pointer); None, None restores hipMalloc / hipFree.  The callbacks are kept
        alive by the context."""
        if alloc is None and release is None:
            self._check(self.lib.seqx_set_allocator(self.h, ALLOC_FN(), RELEASE_FN(), None))
            return
        def _alloc(n, user):
            try:
                return alloc(int(n)) or None
            except Exception:  # reported as a failed allocation (SEQX_E_NOMEM)
                traceback.print_exc()
                return None

        def _release(ptr, user):
            try:
                release(int(ptr))
            except Exception:
                traceback.print_exc()

        cbs = (ALLOC_FN(_alloc), RELEASE_FN(_release))
        if not self._exit_hook:
            # memory must go back through Python callables while the interpreter
            # (and the framework that owns the memory) is still whole
            atexit.register(_close_at_exit, weakref.ref(self))
            self._exit_hook = True
        # buffers made earlier still hand their memory back through the callbacks they
        # were made with, so every pair stays alive as long as the context
        self._callbacks.append(cbs)
        self._check(self.lib.seqx_set_allocator(self.h, cbs[0], cbs[1], None))

    def use_torch_allocator(self, device: int = 0):
        """Route the library's device memory through torch's caching allocator (on the
        current torch stream of `device`)."""
        import torch
        self.set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, device),
                           lambda p: torch.cuda.caching_allocator_delete(p))

    def prepare(self, natoms, Z, xyz, tol=None, max_iter=None, ndiis=None, integrals_only=False) -> "Job":
        natoms = np.ascontiguousarray(np.atleast_1d(natoms), dtype=np.int32)
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        o = ScfOpts(tol or 0.0, max_iter or 0, ndiis or 0, 1 if integrals_only else 0)
        h = C.c_void_p()
        self._check(self.lib.seqx_prepare(self.h, len(natoms), _iptr(natoms), _iptr(Z), _dptr(xyz), C.byref(o),
                                          C.byref(h)))
        return Job(self, h, len(natoms))

    def mlp_set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self.lib.seqx_mlp_set_params(self.h, _fptr(p), p.size))

    def mlp_get_params(self):
        p = np.zeros(MLP_NPARAMS, dtype=np.float32)
        self._check(self.lib.seqx_mlp_get_params(self.h, _fptr(p), p.size, None))
        return p

    def mlp_save(self, path):
        self._check(self.lib.seqx_mlp_save(self.h, os.fsencode(path)))

    def mlp_load(self, path):
        self._check(self.lib.seqx_mlp_load(self.h, os.fsencode(path)))

    def mlp_loss_grad(self, feats, w, seg):
        feats = np.ascontiguousarray(feats, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float32)
        seg = np.ascontiguousarray(seg, dtype=np.int64)
        loss = C.c_double()
        g = np.zeros(MLP_NWEIGHTS, dtype=np.float32)
        self._check(self.lib.seqx_mlp_loss_grad(self.h, w.size, _fptr(feats), _fptr(w), len(seg) - 1,
                                                seg.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(loss), _fptr(g)))
        return loss.value, g

    def broaden(self, omega_eV, f, sigma=0.1, e0=0.0, de=0.01, npts=1000):
        """Gaussian-broadened absorption profile of caller lines (1/eV) on e0 + i de."""
        w = np.ascontiguousarray(omega_eV, dtype=np.float64)
        fv = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(npts)
        self._check(self.lib.seqx_broaden(self.h, w.size, _dptr(w), _dptr(fv), sigma, e0, de, npts, _dptr(out)))
        return out

    def close(self):
        """Free the context's jobs, then the context (seqx_destroy)."""
        if getattr(self, "h", None):
            for job in list(self._jobs):
                job.free()
            self.lib.seqx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _close_at_exit(ref):
    ctx = ref()
    if ctx is not None:
        ctx.close()


class Job:
    def __init__(self, ctx: Context, h, nmol: int):
        self.ctx, self.h, self.nmol = ctx, h, nmol
        self.lib = ctx.lib
        ctx._jobs.add(self)

    def _check(self, s):
        self.ctx._check(s)

    def dims(self, mol=0):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.seqx_dims(self.h, mol, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def scf_results(self, mol=0):
        n, _, _ = self.dims(mol)
        eps, Cm, P = np.zeros(n), np.zeros((n, n)), np.zeros((n, n))
        self._check(self.lib.seqx_scf_results(self.h, mol, _dptr(eps), _dptr(Cm), _dptr(P)))
        return eps, Cm, P

    def core_hamiltonian(self, mol=0):
        n, _, _ = self.dims(mol)
        H = np.zeros((n, n))
        self._check(self.lib.seqx_core_hamiltonian(self.h, mol, _dptr(H)))
        return H

    def integrals(self, mol=0):
        need = C.c_size_t()
        self._check(self.lib.seqx_integrals(self.h, mol, None, 0, C.byref(need)))
        np_ = int(round(need.value ** 0.5))
        W = np.zeros((np_, np_))
        self._check(self.lib.seqx_integrals(self.h, mol, _dptr(W), W.size, C.byref(need)))
        return W

    def sigma(self, V, theory=TDHF, mol=0, precision=FP64):
        """Host arrays V[k, nocc, nvirt] -> (out1, out2) (A V, None) or ((A+B)V, (A-B)V)."""
        V = np.ascontiguousarray(V, dtype=np.float64)
        k = V.shape[0]
        o1 = np.zeros_like(V)
        o2 = np.zeros_like(V) if theory == TDHF else None
        self._check(self.lib.seqx_sigma(self.h, mol, theory, k, _dptr(V), _dptr(o1), _dptr(o2), precision))
        return o1, o2

    def sigma_device(self, V, out1, out2=None, theory=TDHF, mol=0, precision=FP64):
        """torch device tensors (float64, contiguous [k, nocc, nvirt]); ordered on the context stream."""
        k = V.shape[0]
        self._check(self.lib.seqx_sigma_device(self.h, mol, theory, k, C.c_void_p(V.data_ptr()),
                                               C.c_void_p(out1.data_ptr()),
                                               C.c_void_p(out2.data_ptr()) if out2 is not None else None,
                                               precision))

    def sigma_device_noalloc(self, V, out1, out2=None, theory=TDHF, mol=0, precision=FP64):
        """As sigma_device, with the library's fixed per-GPU workspace instead of allocations."""
        k = V.shape[0]
        self._check(self.lib.seqx_sigma_device_noalloc(self.h, mol, theory, k, C.c_void_p(V.data_ptr()),
                                                       C.c_void_p(out1.data_ptr()),
                                                       C.c_void_p(out2.data_ptr()) if out2 is not None else None,
                                                       precision))

    def features(self, mol=0):
        _, o, v = self.dims(mol)
        f = np.zeros((o * v, MLP_NFEAT), dtype=np.float32)
        self._check(self.lib.seqx_features(self.h, mol, _fptr(f), f.size))
        return f

    def mlp_scores(self, mol=0):
        _, o, v = self.dims(mol)
        z = np.zeros(o * v, dtype=np.float32)
        self._check(self.lib.seqx_mlp_scores(self.h, mol, _fptr(z), z.size))
        return z

    def mlp_train(self, epochs=30, batch=32, lr=2e-3, seed=2505, init=True):
        o = TrainOpts(epochs, batch, lr, seed, 1 if init else 0)
        log = TrainLog()
        self._check(self.lib.seqx_mlp_train(self.h, C.byref(o), C.byref(log)))
        return {"loss": list(log.loss[:min(log.n_epochs, 256)]), "seconds": log.seconds}

    def solve(self, theory=TDHF, nroots=3, tol=1e-6, max_iter=100, max_subspace=0, mem_budget_bytes=0,
              precision=FP64, guess=GUESS_GAP, user_guess=None, batched=False, pspace=0, root_batch=0, nguard=0):
        ug = None
        n_ug = 0
        if user_guess is not None:
            ug = np.ascontiguousarray(user_guess, dtype=np.float64)
            n_ug = ug.shape[0]
        o = SolveOpts(theory, nroots, tol, max_iter, max_subspace, mem_budget_bytes, precision, guess, n_ug,
                      _dptr(ug) if ug is not None else None, 1 if batched else 0, pspace, root_batch, nguard)
        self.nroots = 0
        self._check(self.lib.seqx_solve(self.h, C.byref(o)))
        self.nroots = nroots

    def results(self, mol=0) -> Results:
        _, o, v = self.dims(mol)
        K = getattr(self, "nroots", 0)
        om, f, mu = np.zeros(K), np.zeros(K), np.zeros((K, 3))
        X, Y = np.zeros((K, o, v)), np.zeros((K, o, v))
        self._check(self.lib.seqx_results(self.h, mol, _dptr(om), _dptr(X), _dptr(Y), _dptr(f), _dptr(mu)))
        return Results(om, X, Y, f, mu)

    def param_gradient(self, mol=0):
        """d omega / d theta [K, 3 (H, C, O), NPARAM] in eV per parameter unit, and the Z-vector iterations."""
        K = getattr(self, "nroots", 0)
        g = np.zeros((K, 3, NPARAM))
        it = C.c_int32()
        self._check(self.lib.seqx_param_gradient(self.h, mol, _dptr(g), g.size, C.byref(it)))
        return g, it.value

    def spectrum(self, mol=0, sigma=0.1, e0=0.0, de=0.01, npts=1000):
        """Gaussian-broadened absorption profile (1/eV) of the solved roots on e0 + i de."""
        out = np.zeros(npts)
        self._check(self.lib.seqx_spectrum(self.h, mol, sigma, e0, de, npts, _dptr(out)))
        return out

    def history(self, mol=0):
        """(t_s[iterations], omega_eV[iterations, K]) of the last solve."""
        n = C.c_int32()
        self._check(self.lib.seqx_history(self.h, mol, 0, C.byref(n), None, None))
        K = getattr(self, "nroots", 0)
        t = np.zeros(n.value)
        om = np.zeros((n.value, K))
        self._check(self.lib.seqx_history(self.h, mol, n.value, C.byref(n), _dptr(t), _dptr(om)))
        return t, om

    def stats(self) -> Stats:
        s = Stats()
        self._check(self.lib.seqx_get_stats(self.h, C.byref(s)))
        return s

    def free(self):
        if getattr(self, "h", None):
            self.lib.seqx_job_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def params_table(params: dict):
    """{Z: {name: value}} (eV, 1/bohr) -> (Z[nel], values[nel, 11]) in the ABI's parameter order."""
    names = ["zeta_s", "zeta_p", "U_ss", "U_pp", "beta_s", "beta_p", "g_ss", "g_sp", "g_pp", "g_p2", "h_sp"]
    Zs = sorted(params)
    vals = np.zeros((len(Zs), NPARAM))
    for r, z in enumerate(Zs):
        for c, nm in enumerate(names):
            vals[r, c] = params[z].get(nm, 0.0)
    return np.array(Zs, dtype=np.int32), vals
