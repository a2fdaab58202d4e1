"""ctypes declarations of include/dmrg_mi355x.h and small owning wrappers."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # torch first: the library then binds to the HIP runtime torch already loaded
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for host-only use
    torch = None

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdmrg_mi355x.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_09990_amd.build` "
                      "(there is no CPU fallback)")
lib = C.CDLL(LIB_PATH)

_p, _i, _d, _i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64


class dmrg_options(C.Structure):
    _fields_ = [("M", C.c_int), ("n_states", C.c_int), ("weights", C.POINTER(C.c_double)),
                ("davidson_tol", C.c_double), ("max_iter", C.c_int), ("max_subspace", C.c_int),
                ("precision", C.c_int), ("precond", C.c_int), ("seed", C.c_ulonglong),
                ("tie_rtol", C.c_double), ("cut_rtol", C.c_double), ("verbose", C.c_int),
                ("sigma_chunk_bytes", C.c_longlong), ("pcg_steps", C.c_int), ("pcg_rtol", C.c_double),
                ("trunc_tol", C.c_double), ("m_min", C.c_int)]


def _decl(name, args, res=C.c_int):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


dmrg_options_default = _decl("dmrg_options_default", [C.POINTER(dmrg_options)], None)
dmrg_problem_create = _decl("dmrg_problem_create", [_i, _i, _i, _i, _p, _p, _d, C.POINTER(_p)])
dmrg_problem_destroy = _decl("dmrg_problem_destroy", [_p], None)
dmrg_mpo_dims = _decl("dmrg_mpo_dims", [_p, _p])
dmrg_mpo_site_nnz = _decl("dmrg_mpo_site_nnz", [_p, _i, C.POINTER(_i)])
dmrg_mpo_site = _decl("dmrg_mpo_site", [_p, _i, _p, _p, _p, _p])
dmrg_solver_create = _decl("dmrg_solver_create", [_p, C.POINTER(dmrg_options), _p, C.POINTER(_p)])
dmrg_solver_destroy = _decl("dmrg_solver_destroy", [_p], None)
dmrg_set_mps = _decl("dmrg_set_mps", [_p, _p, _p, _p])
dmrg_get_bonds = _decl("dmrg_get_bonds", [_p, _p, _p, _i])
dmrg_prepare = _decl("dmrg_prepare", [_p, _i, C.POINTER(_i64)])
dmrg_sigma = _decl("dmrg_sigma", [_p, _i, _i, _i64, _p, _p, C.POINTER(_d)])
dmrg_diag = _decl("dmrg_diag", [_p, _i, _i64, _p])
dmrg_workspace_query = _decl("dmrg_workspace_query", [_p, C.POINTER(C.c_size_t)])
dmrg_workspace_attach = _decl("dmrg_workspace_attach", [_p, _p, C.c_size_t])
dmrg_export_mps = _decl("dmrg_export_mps", [_p, _p, _p, _i, _p, _i64, C.POINTER(_i64)])
dmrg_truncate = _decl("dmrg_truncate", [_p, _i, _i, _i64, _p, C.POINTER(_d), _p, _i, C.POINTER(_i)])
dmrg_sweep = _decl("dmrg_sweep", [_p, _i, _p, C.POINTER(_d)])
dmrg_energy = _decl("dmrg_energy", [_p, _p])
dmrg_deflate_add = _decl("dmrg_deflate_add", [_p, _p, _p, _p, _d])
dmrg_deflate_clear = _decl("dmrg_deflate_clear", [_p])
dmrg_deflate_project = _decl("dmrg_deflate_project", [_p, _i, _i, _i64, _p])
dmrg_overlap = _decl("dmrg_overlap", [_p, _i, C.POINTER(_d)])
dmrg_s_squared = _decl("dmrg_s_squared", [_p, _p])
dmrg_step = _decl("dmrg_step", [_p, _i, _i, _p, C.POINTER(_d)])
dmrg_set_kernel_tag = _decl("dmrg_set_kernel_tag", [_p, _i])
dmrg_get_stats = _decl("dmrg_get_stats", [_p, _p, _i])
dmrg_block_gemm = _decl("dmrg_block_gemm", [_i, _i, _i, _i, _i, _p, _i, _p, _i, _p, _i, _d, _p])
dmrg_block_gemm_noalloc = _decl("dmrg_block_gemm_noalloc", [_i, _i, _i, _i, _i, _p, _i, _p, _i, _p, _i, _d, _p])
dmrg_measure_peaks = _decl("dmrg_measure_peaks", [_p, _p, _p, C.c_size_t, _p, _p])
dmrg_get_env = _decl("dmrg_get_env", [_p, _i, _i, _p, _i64, C.POINTER(_i64)])
dmrg_grad = _decl("dmrg_grad", [_p, _p, _p, _p, _p])
dmrg_mlp_create = _decl("dmrg_mlp_create", [_i, _i, C.c_ulonglong, _p, C.POINTER(_p)])
dmrg_mlp_destroy = _decl("dmrg_mlp_destroy", [_p], None)
dmrg_mlp_num_params = _decl("dmrg_mlp_num_params", [_p, C.POINTER(_i64)])
dmrg_mlp_set_params = _decl("dmrg_mlp_set_params", [_p, _p, _i64])
dmrg_mlp_get_params = _decl("dmrg_mlp_get_params", [_p, _p, _i64])
dmrg_mlp_forward = _decl("dmrg_mlp_forward", [_p, _i, _p, _i64, _p])
dmrg_mlp_loss_grad = _decl("dmrg_mlp_loss_grad", [_p, _p, _p, _i, _i, C.POINTER(_d), _p])
dmrg_mlp_adam_step = _decl("dmrg_mlp_adam_step", [_p, _d])
dmrg_set_precond = _decl("dmrg_set_precond", [_p, _i, _p])
dmrg_set_precision = _decl("dmrg_set_precision", [_p, _i])
dmrg_record_triples = _decl("dmrg_record_triples", [_p, _i, _i])
dmrg_take_triples = _decl("dmrg_take_triples", [_p, _p, _p, _i, C.POINTER(_i)])
dmrg_precond_features = _decl("dmrg_precond_features", [_p, _i, _i64, _p, _p, _d, _p])
dmrg_correction = _decl("dmrg_correction", [_p, _i, _i, _i64, _p, _p, _p, _d, _p, _p])
dmrg_stationarize = _decl("dmrg_stationarize", [_p, _i, _p, _p])
dmrg_orbital_rdm2 = _decl("dmrg_orbital_rdm2", [_p, _i64, _p, _p, _p])
dmrg_ci_apply_v = _decl("dmrg_ci_apply_v", [_p, _i64, _p, _p, _p])
dmrg_ci_rdm3 = _decl("dmrg_ci_rdm3", [_p, _i64, _p, _p, _p, _p])
dmrg_mutual_information = _decl("dmrg_mutual_information", [_p, _i64, _p, _p, _p, _p])
dmrg_fiedler_order = _decl("dmrg_fiedler_order", [_i, _p, _p, _p])
dmrg_mps_orbital_rdm2 = _decl("dmrg_mps_orbital_rdm2", [_p, _p, _p, _p])
dmrg_ci_dims = _decl("dmrg_ci_dims", [_p, _p, _p])
dmrg_mps_to_ci = _decl("dmrg_mps_to_ci", [_p, _i, _p, _i64])
dmrg_ci_rdm12 = _decl("dmrg_ci_rdm12", [_p, _i64, _p, _p, _p, _p, _p, _p])
dmrg_rdm12 = _decl("dmrg_rdm12", [_p, _i, _i, _p, _p, _p])
dmrg_last_error = _decl("dmrg_last_error", [], C.c_char_p)

STATUS = {0: "DMRG_OK", -1: "DMRG_EINVAL", -2: "DMRG_ENOMEM", -3: "DMRG_EHIP", -4: "DMRG_ENOCONV",
          -5: "DMRG_ESECTOR", -6: "DMRG_ESTATE"}


class DMRGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise DMRGError(code, (dmrg_last_error() or b"").decode())


def _ptr(a):
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


class Problem:
    """dmrg_problem: active-space integrals and the MPO built from them (host)."""

    def __init__(self, h, B, n_alpha, n_beta, e_core=0.0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        n = h.shape[0]
        nq = B.shape[0] if B.ndim == 3 else 0
        self.n, self.n_alpha, self.n_beta, self.n_chol = n, n_alpha, n_beta, nq
        self._keep = (h, B)
        self.h = C.c_void_p()
        _check(dmrg_problem_create(n, n_alpha, n_beta, nq, _ptr(h), _ptr(B), float(e_core),
                                   C.byref(self.h)))

    def mpo_dims(self):
        d = np.zeros(self.n + 1, dtype=np.int32)
        _check(dmrg_mpo_dims(self.h, _ptr(d)))
        return d

    def ci_dims(self):
        """(C(n, n_alpha), C(n, n_beta)): the CI matrix shape."""
        a, b = C.c_int64(), C.c_int64()
        _check(dmrg_ci_dims(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def ci_rdm12(self, bra, ket=None, stream=None):
        """Unnormalised (transition) 1-/2-RDMs of device CI vectors: (gamma[n, n],
        Gamma[n, n, n, n], <bra|ket>), gamma_pq = <bra|E_pq|ket>, Gamma_pqrs =
        <bra|E_pq E_rs|ket> - d_qr gamma_ps."""
        ket = bra if ket is None else ket
        na, nb = self.ci_dims()
        Solver._dev_f64(bra, "bra", na * nb)
        Solver._dev_f64(ket, "ket", na * nb)
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        n = self.n
        g, G, o = np.zeros((n, n)), np.zeros((n, n, n, n)), C.c_double()
        _check(dmrg_ci_rdm12(self.h, na * nb, _ptr(bra), _ptr(ket), _ptr(g), _ptr(G), C.byref(o), stream))
        return g, G, o.value

    def ci_apply_v(self, c, out=None, stream=None):
        """V c, V = 1/2 sum (pq|rs) E_pq E_rs (device CI vectors)."""
        na, nb = self.ci_dims()
        Solver._dev_f64(c, "c", na * nb)
        if out is None:
            out = torch.empty_like(c)
        Solver._dev_f64(out, "out", na * nb)
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(dmrg_ci_apply_v(self.h, na * nb, _ptr(c), _ptr(out), stream))
        return out

    def ci_rdm3(self, bra, ket=None, stream=None):
        """<bra|E_pq E_rs E_tu|ket> (unnormalised) as a host array [n]*6."""
        ket = bra if ket is None else ket
        na, nb = self.ci_dims()
        Solver._dev_f64(bra, "bra", na * nb)
        Solver._dev_f64(ket, "ket", na * nb)
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        n = self.n
        out = np.zeros((n,) * 6)
        _check(dmrg_ci_rdm3(self.h, na * nb, _ptr(bra), _ptr(ket), _ptr(out), stream))
        return out

    def orbital_rdm2(self, c, stream=None):
        """Two-orbital density matrices of a device CI vector: [n(n-1)/2, 16, 16]."""
        na, nb = self.ci_dims()
        Solver._dev_f64(c, "c", na * nb)
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        n = self.n
        rho = np.zeros((n * (n - 1) // 2, 16, 16))
        _check(dmrg_orbital_rdm2(self.h, na * nb, _ptr(c), _ptr(rho), stream))
        return rho

    def mutual_information(self, c, stream=None):
        """(one-orbital entropies s1[n], mutual information I[n, n]) of a device CI vector."""
        na, nb = self.ci_dims()
        Solver._dev_f64(c, "c", na * nb)
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        n = self.n
        s1, I = np.zeros(n), np.zeros((n, n))
        _check(dmrg_mutual_information(self.h, na * nb, _ptr(c), _ptr(s1), _ptr(I), stream))
        return s1, I

    def mpo_site(self, k):
        nnz = C.c_int()
        _check(dmrg_mpo_site_nnz(self.h, k, C.byref(nnz)))
        m = nnz.value
        a = np.zeros(m, np.int32)
        b = np.zeros(m, np.int32)
        c = np.zeros(m)
        op = np.zeros((m, 16))
        _check(dmrg_mpo_site(self.h, k, _ptr(a), _ptr(b), _ptr(c), _ptr(op)))
        return a, b, c, op.reshape(m, 4, 4)

    def __del__(self):
        if getattr(self, "h", None) and dmrg_problem_destroy is not None:
            dmrg_problem_destroy(self.h)
            self.h = None


class MLP:
    """dmrg_mlp: the preconditioner network (parameters on the device)."""

    def __init__(self, n_in=8, width=256, seed=0, stream=None):
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.n_in, self.width = n_in, width
        self.h = C.c_void_p()
        _check(dmrg_mlp_create(n_in, width, seed, C.c_void_p(stream or 0), C.byref(self.h)))
        n = C.c_int64()
        _check(dmrg_mlp_num_params(self.h, C.byref(n)))
        self.n_params = n.value

    def params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(dmrg_mlp_get_params(self.h, _ptr(p), self.n_params))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(dmrg_mlp_set_params(self.h, _ptr(p), p.size))

    def unpack(self, p=None):
        """Parameter vector as {W1, b1, W2, b2, W3, b3} views (host)."""
        p = self.params() if p is None else p
        F, W = self.n_in, self.width
        out, o = {}, 0
        for k, shape in (("W1", (W, F)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (1, W)), ("b3", (1,))):
            size = int(np.prod(shape))
            out[k] = p[o:o + size].reshape(shape)
            o += size
        return out

    @staticmethod
    def pack(P):
        return np.concatenate([np.asarray(P[k], dtype=np.float32).ravel()
                               for k in ("W1", "b1", "W2", "b2", "W3", "b3")])

    def forward(self, X, y, precision=1):
        _check(dmrg_mlp_forward(self.h, precision, _ptr(X), X.shape[0], _ptr(y)))

    def loss_grad(self, X, T, n_seg, seg_len, want_grad=False):
        loss = C.c_double()
        g = np.zeros(self.n_params, dtype=np.float32) if want_grad else None
        _check(dmrg_mlp_loss_grad(self.h, _ptr(X), _ptr(T), n_seg, seg_len, C.byref(loss),
                                  None if g is None else _ptr(g)))
        return (loss.value, g) if want_grad else loss.value

    def adam_step(self, lr):
        _check(dmrg_mlp_adam_step(self.h, lr))

    def __del__(self):
        if getattr(self, "h", None):
            dmrg_mlp_destroy(self.h)
            self.h = None


class Solver:
    """dmrg_solver on the current device; device arrays are torch tensors."""

    def __init__(self, problem: Problem, M=256, n_states=1, weights=None, tol=1e-10, max_iter=200,
                 max_subspace=32, precision=0, precond=0, seed=1, tie_rtol=1e-10, cut_rtol=1e-14,
                 verbose=0, stream=None, workspace=False, sigma_chunk_bytes=0, pcg_steps=5, pcg_rtol=0.1,
                 trunc_tol=0.0, m_min=1):
        """workspace: False (the library allocates its device buffers), True (a
        torch-allocated workspace of dmrg_workspace_query bytes, grown and
        re-attached when a call reports DMRG_ENOMEM) or a byte count."""
        o = dmrg_options()
        dmrg_options_default(C.byref(o))
        o.M, o.n_states, o.davidson_tol, o.max_iter = M, n_states, tol, max_iter
        o.max_subspace, o.precision, o.precond, o.seed = max_subspace, precision, precond, seed
        o.tie_rtol, o.cut_rtol, o.verbose = tie_rtol, cut_rtol, verbose
        o.sigma_chunk_bytes = int(sigma_chunk_bytes)
        o.pcg_steps, o.pcg_rtol = int(pcg_steps), float(pcg_rtol)
        o.trunc_tol, o.m_min = float(trunc_tol), int(m_min)
        self._w = None
        if weights is not None:
            self._w = np.ascontiguousarray(weights, dtype=np.float64)
            o.weights = self._w.ctypes.data_as(C.POINTER(C.c_double))
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.problem = problem
        self.n_states = n_states
        self.h = C.c_void_p()
        _check(dmrg_solver_create(problem.h, C.byref(o), C.c_void_p(stream or 0), C.byref(self.h)))
        self._ws = None
        if workspace:
            self.attach_workspace(None if workspace is True else int(workspace))

    def workspace_query(self):
        b = C.c_size_t()
        _check(dmrg_workspace_query(self.h, C.byref(b)))
        return b.value

    def attach_workspace(self, nbytes=None):
        """Allocate a device workspace with torch (nbytes, default the queried
        size) and hand it to the library; the previous one is released after."""
        nbytes = self.workspace_query() if nbytes is None else nbytes
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(dmrg_workspace_attach(self.h, C.c_void_p(buf.data_ptr()), nbytes))
        self._ws = buf
        return nbytes

    def _grow(self, fn):
        """Run fn(); with a torch workspace, a DMRG_ENOMEM re-attaches a larger one and runs it again."""
        try:
            return fn()
        except DMRGError as e:
            if e.code != -2 or self._ws is None:
                raise
            self.attach_workspace()
            return fn()

    def set_mps(self, bonds, sites):
        n_sec = np.array([len(b) for b in bonds], dtype=np.int32)
        sec = np.array([x for b in bonds for s in b for x in s], dtype=np.int32)
        data = np.ascontiguousarray(np.concatenate(sites), dtype=np.float64)
        _check(dmrg_set_mps(self.h, _ptr(n_sec), _ptr(sec), _ptr(data)))

    def bonds(self):
        n_sec = np.zeros(self.problem.n + 1, dtype=np.int32)
        cap = 1 << 16
        sec = np.zeros(3 * cap, dtype=np.int32)
        _check(dmrg_get_bonds(self.h, _ptr(n_sec), _ptr(sec), cap))
        out, i = [], 0
        for c in range(self.problem.n + 1):
            out.append([tuple(int(v) for v in sec[3 * j:3 * j + 3]) for j in range(i, i + n_sec[c])])
            i += n_sec[c]
        return out

    def prepare(self, k):
        n = C.c_int64()
        self._grow(lambda: _check(dmrg_prepare(self.h, k, C.byref(n))))
        return n.value

    @staticmethod
    def _dev_f64(t, name, numel=None):
        """Device kernels take raw pointers: refuse anything but a contiguous
        float64 tensor on the GPU (of numel elements when given)."""
        if torch is None or not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor on the GPU")
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor "
                            f"(got {t.dtype}, device {t.device}, contiguous {t.is_contiguous()})")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")

    def sigma(self, k, psi, out, precision=0):
        """out = H_eff psi for step k; returns the executed flops."""
        self._dev_f64(psi, "psi")
        self._dev_f64(out, "out", psi.numel())
        fl = C.c_double()
        self._grow(lambda: _check(dmrg_sigma(self.h, k, precision, psi.numel(), _ptr(psi), _ptr(out), C.byref(fl))))
        return fl.value

    def diag(self, k, out):
        self._dev_f64(out, "out")
        self._grow(lambda: _check(dmrg_diag(self.h, k, out.numel(), _ptr(out))))

    def export_mps(self):
        """The current MPS as {bonds: [[(N, 2Sz, dim), ...] per cut], sites: [flat float64 per site]}."""
        L = self.problem.n
        n_sec = np.zeros(L + 1, dtype=np.int32)
        size = C.c_int64()
        _check(dmrg_export_mps(self.h, _ptr(n_sec), None, 0, None, 0, C.byref(size)))
        tot = int(n_sec.sum())
        sec = np.zeros(3 * tot, dtype=np.int32)
        data = np.zeros(size.value)
        _check(dmrg_export_mps(self.h, _ptr(n_sec), _ptr(sec), tot, _ptr(data), size.value, C.byref(size)))
        bonds, i = [], 0
        for c in range(L + 1):
            bonds.append([tuple(int(v) for v in sec[3 * j:3 * j + 3]) for j in range(i, i + n_sec[c])])
            i += n_sec[c]
        sites, off = [], 0
        for k in range(L):
            sz = _slab_size(bonds[k], bonds[k + 1])
            sites.append(data[off:off + sz].copy())
            off += sz
        assert off == size.value
        return {"bonds": bonds, "sites": sites}

    def truncate(self, k, psi, direction=0, sv_cap=1 << 20):
        """dmrg_truncate on device vectors psi (n_states x n, root-major, contiguous):
        returns (tau, kept singular values descending)."""
        self._dev_f64(psi, "psi")
        if psi.numel() % self.n_states:
            raise ValueError("psi must hold n_states vectors")
        n = psi.numel() // self.n_states
        tau = C.c_double()
        nk = C.c_int()
        sv = np.zeros(sv_cap)
        _check(dmrg_truncate(self.h, k, direction, n, _ptr(psi), C.byref(tau), _ptr(sv), sv_cap, C.byref(nk)))
        return tau.value, sv[:min(nk.value, sv_cap)].copy()

    def sweep(self, n_sweeps=1):
        e = np.zeros(self.n_states)
        tau = C.c_double()
        code = dmrg_sweep(self.h, n_sweeps, _ptr(e), C.byref(tau))
        if code not in (0, -4):
            _check(code)
        return e, tau.value, code == 0

    def stationarize(self, n_sweeps=1):
        """One-site sweeps at the current bond dimensions: (energy, largest local
        tangent gradient of the last sweep, converged)."""
        e, r = C.c_double(), C.c_double()
        code = dmrg_stationarize(self.h, n_sweeps, C.byref(e), C.byref(r))
        if code not in (0, -4):
            _check(code)
        return e.value, r.value, code == 0

    def step(self, k, direction=0):
        e = np.zeros(self.n_states)
        tau = C.c_double()

        def run():
            code = dmrg_step(self.h, k, direction, _ptr(e), C.byref(tau))
            if code not in (0, -4):
                _check(code)
            return code
        code = self._grow(run)
        return e, tau.value, code == 0

    def set_precision(self, precision):
        _check(dmrg_set_precision(self.h, precision))

    def set_precond(self, precond, net=None):
        """0: diagonal, 1: learned with the MLP `net` (kept alive by this object),
        2: Olsen, 3: shift-and-invert inner PCG."""
        self._net = net
        _check(dmrg_set_precond(self.h, precond, net.h if net is not None else None))

    def record_triples(self, capacity, sample):
        self._sample = sample
        _check(dmrg_record_triples(self.h, capacity, sample))

    def take_triples(self, X, T, cap):
        cnt = C.c_int()
        _check(dmrg_take_triples(self.h, _ptr(X), _ptr(T), cap, C.byref(cnt)))
        return cnt.value

    def features(self, k, r, d, theta, X):
        self._dev_f64(r, "r")
        self._dev_f64(d, "d", r.numel())
        if not (X.is_cuda and X.dtype == torch.float32 and X.is_contiguous() and X.numel() == 8 * r.numel()):
            raise TypeError("X must be a contiguous float32 CUDA tensor of 8 n elements")
        _check(dmrg_precond_features(self.h, k, r.numel(), _ptr(r), _ptr(d), float(theta), _ptr(X)))

    def correction(self, k, mode, x, r, d, theta, t):
        """One correction of the preconditioner family into device t; returns the
        sigma products it made."""
        self._dev_f64(x, "x")
        for v, name in ((r, "r"), (d, "d"), (t, "t")):
            self._dev_f64(v, name, x.numel())
        mv = C.c_int()
        _check(dmrg_correction(self.h, k, mode, x.numel(), _ptr(x), _ptr(r), _ptr(d), float(theta), _ptr(t),
                               C.byref(mv)))
        return mv.value

    def set_kernel_tag(self, tag):
        _check(dmrg_set_kernel_tag(self.h, tag))

    def energy(self):
        e = np.zeros(self.n_states)
        _check(dmrg_energy(self.h, _ptr(e)))
        return e

    def deflate(self, mps, weight):
        """Hold a lower state (an export_mps dict of the same problem) for penalty
        deflation with the given weight (Ha); later solves see H + w |Phi><Phi|."""
        n_sec = np.array([len(b) for b in mps["bonds"]], dtype=np.int32)
        sec = np.array([x for b in mps["bonds"] for s in b for x in s], dtype=np.int32)
        data = np.ascontiguousarray(np.concatenate(mps["sites"]), dtype=np.float64)
        self._grow(lambda: _check(dmrg_deflate_add(self.h, _ptr(n_sec), _ptr(sec), _ptr(data), float(weight))))

    def clear_deflation(self):
        _check(dmrg_deflate_clear(self.h))

    def mps_to_ci(self, state=0, out=None):
        """CI matrix [C(n, n_alpha), C(n, n_beta)] (device float64) of this MPS
        (state 0) or of held state `state` (1..), as stored."""
        na, nb = self.problem.ci_dims()
        if out is None:
            out = torch.empty((na, nb), dtype=torch.float64, device="cuda")
        self._dev_f64(out, "out", na * nb)
        self._grow(lambda: _check(dmrg_mps_to_ci(self.h, state, _ptr(out), na * nb)))
        return out

    def rdm12(self, bra=0, ket=None):
        """Normalised (transition) 1-/2-RDMs of MPS states (0: this MPS, j >= 1:
        held state j-1): (gamma[n, n], Gamma[n, n, n, n], overlap)."""
        ket = bra if ket is None else ket
        n = self.problem.n
        g, G, o = np.zeros((n, n)), np.zeros((n, n, n, n)), C.c_double()
        self._grow(lambda: _check(dmrg_rdm12(self.h, bra, ket, _ptr(g), _ptr(G), C.byref(o))))
        return g, G, o.value

    def orbital_entanglement(self):
        """(two-orbital density matrices [n(n-1)/2, 16, 16], s1[n], I[n, n]) of the
        MPS as stored, from the MPS itself (no CI vector)."""
        n = self.problem.n
        rho, s1, I = np.zeros((n * (n - 1) // 2, 16, 16)), np.zeros(n), np.zeros((n, n))
        self._grow(lambda: _check(dmrg_mps_orbital_rdm2(self.h, _ptr(rho), _ptr(s1), _ptr(I))))
        return rho, s1, I

    def deflate_project(self, k, j, out):
        """Projection of lower state j into step k's two-site space (device out)."""
        self._dev_f64(out, "out")
        self._grow(lambda: _check(dmrg_deflate_project(self.h, k, j, out.numel(), _ptr(out))))

    def overlap(self, j):
        """Normalised <Psi|Phi_j> of the current MPS with lower state j (fp64)."""
        v = C.c_double()
        self._grow(lambda: _check(dmrg_overlap(self.h, j, C.byref(v))))
        return v.value

    def s_squared(self):
        """Per-root <S^2> of the current MPS (centre on site 0, i.e. after a sweep)."""
        v = np.zeros(self.n_states)
        self._grow(lambda: _check(dmrg_s_squared(self.h, _ptr(v))))
        return v

    def env(self, cut, side):
        """Environment arrays of the current MPS (side 0 left, 1 right), host copy."""
        n = C.c_int64()
        _check(dmrg_get_env(self.h, cut, side, None, 0, C.byref(n)))
        out = np.zeros(n.value)
        _check(dmrg_get_env(self.h, cut, side, _ptr(out), n.value, C.byref(n)))
        return out

    def grad(self, weights=None):
        """dmrg_grad: (sum_r w_r dE_r/dh, sum_r w_r dE_r/dB, energies) as host arrays."""
        p = self.problem
        dh = np.zeros((p.n, p.n))
        dB = np.zeros((max(p.n_chol, 0), p.n, p.n))
        e = np.zeros(self.n_states)
        w = None
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            if w.shape != (self.n_states,):
                raise ValueError(f"weights must have shape ({self.n_states},)")
        _check(dmrg_grad(self.h, None if w is None else _ptr(w), _ptr(dh),
                         _ptr(dB) if p.n_chol > 0 else None, _ptr(e)))
        return dh, dB, e

    def rdm1(self):
        """The spin-summed 1-RDM gamma_pq = <E_pq> of the MPS as stored (root 0),
        from the MPS itself at any size: it is dE/dh of dmrg_grad."""
        dh, _, _ = self.grad()
        return dh

    def stats(self):
        s = np.zeros(30)
        _check(dmrg_get_stats(self.h, _ptr(s), 30))
        keys = ["matvecs", "davidson_iters", "sigma_ms", "env_ms", "svd_ms", "sigma_flops", "tau",
                "max_bond", "fallbacks", "converged", "sigma_a_ms", "sigma_b_ms", "sigma_a_flops",
                "sigma_b_flops", "env_flops", "refinements", "sigma_b_gemm_ms", "grad_ms", "grad_flops",
                "prepare_ms", "resolve_ms", "davidson_ms", "plan_hits", "sigma_a_flops_exec",
                "sigma_b_flops_exec", "lowp_matvecs", "workspace_peak_bytes", "device_allocs_since_attach",
                "plan_build_ms", "env_plan_ms"]
        return dict(zip(keys, s.tolist()))

    def __del__(self):
        if getattr(self, "h", None) and dmrg_solver_destroy is not None:
            dmrg_solver_destroy(self.h)
            self.h = None


_SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _slab_size(bond_l, bond_r):
    """Doubles of a site tensor in slab layout between two bonds."""
    right = {(N, s): d for N, s, d in bond_r}
    size = 0
    for N, s, ml in bond_l:
        size += ml * sum(right.get((N + dn, s + ds), 0) for dn, ds in _SITE_QN)
    return size


def measure_peaks(nbytes=1 << 31, stream=None):
    """dmrg_measure_peaks on two torch device buffers of nbytes each:
    (fp64 MFMA TFLOP/s of a register-only loop, streaming-copy GB/s)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    f, c = C.c_double(), C.c_double()
    _check(dmrg_measure_peaks(C.c_void_p(st), C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                              nbytes, C.byref(f), C.byref(c)))
    del src, dst
    return f.value, c.value


def fiedler_order(I):
    """Orbital order (new orbital t = old order[t]) and the Fiedler vector of a
    mutual-information matrix (dmrg_fiedler_order)."""
    I = np.ascontiguousarray(I, dtype=np.float64)
    n = I.shape[0]
    order, v = np.zeros(n, dtype=np.int32), np.zeros(n)
    _check(dmrg_fiedler_order(n, _ptr(I), _ptr(order), _ptr(v)))
    return order, v


def reorder_integrals(h, B, order):
    """h and B^Q in the orbital order `order` (new orbital t = old order[t])."""
    o = np.asarray(order)
    return np.ascontiguousarray(h[np.ix_(o, o)]), np.ascontiguousarray(B[:, o][:, :, o])
