"""Python binding of libcprand (randomized CP-ALS for gfx950).

Argument marshalling only: every function here has the name of a C entry
point of include/cprand.h, takes torch tensors that already live on the GPU,
passes their pointers and the current HIP stream, and raises on a negative
status.  No arithmetic of the method happens in Python; if the library is not
built the import fails.

Layout conventions (see include/cprand.h): a tensor is described by a
`View` (flat device buffer + dims + strides in elements, column-major by
default); factors are row-major (I_m, R) torch tensors.
"""
import ctypes as C
import math

import torch

from . import _abi
from ._abi import (BF16, C64, C128, EHIP, EINVAL, ENAN, ENOMEM, EUNSUPPORTED, F32, F64, MIX_DCT, MIX_FFT,
                   MIX_NONE, OK, PREC_BF16, PREC_BF16_REFINE, PREC_NATIVE, PROPOSAL_LEARNED,
                   PROPOSAL_LEVERAGE, PROPOSAL_MARGINAL, PROPOSAL_MIXTURE, PROPOSAL_TABLE, PROPOSAL_UNIFORM, W_FALLBACK,
                   W_MAXIT, W_PINV)

_lib = _abi.load()

_DTYPES = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16,
           torch.complex64: C64, torch.complex128: C128}


class CprandError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("cprand error %d (%s): %s" % (code, _lib.cprand_strerror(code).decode(), msg))
        self.code = code


def _check(rc):
    if rc < 0:
        raise CprandError(rc, _lib.cprand_last_error().decode())
    return rc


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _ptr_array(ts, order):
    arr = (C.c_void_p * order)()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def colmajor_strides(dims):
    s, out = 1, []
    for d in dims:
        out.append(s)
        s *= d
    return out


class View:
    """A tensor as the C ABI sees it: buffer + dims + strides (elements)."""

    def __init__(self, data, dims, strides=None, dtype=None):
        self.data = data
        self.dims = tuple(int(d) for d in dims)
        self.strides = tuple(int(s) for s in (strides or colmajor_strides(self.dims)))
        self.dtype = _DTYPES[data.dtype] if dtype is None else dtype

    def c(self):
        t = _abi.cprand_tensor()
        t.order = len(self.dims)
        t.dtype = self.dtype
        for i, (d, s) in enumerate(zip(self.dims, self.strides)):
            t.dims[i] = d
            t.strides[i] = s
        t.data = self.data.data_ptr()
        return t


def cprand_version():
    return _lib.cprand_version().decode()


def cprand_workspace_size(X, R, S, P_hat=0):
    return int(_lib.cprand_workspace_size(C.byref(X.c()), R, S, P_hat))


def workspace(X, R, S, P_hat=0):
    n = cprand_workspace_size(X, R, S, P_hat)
    if n == 0:
        raise CprandError(EINVAL, "invalid sizes for a workspace")
    return torch.empty(n, dtype=torch.uint8, device=X.data.device)


def cprand_sample(dims, n, S, seed, t, cdf=None, idx=None, w=None, device="cuda"):
    order = len(dims)
    if idx is None:
        idx = torch.empty((S, order), dtype=torch.int32, device=device)
    if w is None and cdf is not None:
        w = torch.empty(S, dtype=torch.float64, device=device)
    cdims = (C.c_int64 * order)(*dims)
    carr = None
    if cdf is not None:
        carr = _ptr_array([None if m == n else cdf[m] for m in range(order)], order)
    _check(_lib.cprand_sample(order, cdims, n, S, C.c_uint64(seed), C.c_uint64(t), carr, _ptr(idx), _ptr(w),
                              _stream()))
    return idx, w


def cprand_mttkrp_sampled(X, n, A, R, S, idx, w=None, unmix_signs=None, W=None, V=None, ws=None):
    order = len(X.dims)
    real = torch.float64 if X.dtype in (F64, C128) else torch.float32
    if W is None:
        W = torch.empty((X.dims[n], R), dtype=real, device=X.data.device)
    if V is None:
        V = torch.empty((R, R), dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = workspace(X, R, S)
    arr = _ptr_array([None if m == n else A[m] for m in range(order)], order)
    _check(_lib.cprand_mttkrp_sampled(C.byref(X.c()), n, arr, R, S, _ptr(idx), _ptr(w), _ptr(unmix_signs),
                                      _ptr(W), _ptr(V), _ptr(ws), ws.numel(), _stream()))
    return W, V


def cprand_mttkrp_sampled_noalloc(X, n, A, R, S, idx, w=None, W=None, V=None):
    """cprand_mttkrp_sampled with the library's fixed scratch array instead of
    a workspace (real tensors only)."""
    order = len(X.dims)
    real = torch.float64 if X.dtype == F64 else torch.float32
    if W is None:
        W = torch.empty((X.dims[n], R), dtype=real, device=X.data.device)
    if V is None:
        V = torch.empty((R, R), dtype=torch.float64, device=X.data.device)
    arr = _ptr_array([None if m == n else A[m] for m in range(order)], order)
    _check(_lib.cprand_mttkrp_sampled_noalloc(C.byref(X.c()), n, arr, R, S, _ptr(idx), _ptr(w), _ptr(W), _ptr(V),
                                              _stream()))
    return W, V


def cprand_solve(V, W, W_refine=None, V_refine=None, A_out=None, lambda_out=None, info=None, ws=None):
    In, R = W.shape
    dtype = F64 if W.dtype == torch.float64 else F32
    if A_out is None:
        A_out = torch.empty_like(W)
    if lambda_out is None:
        lambda_out = torch.empty(R, dtype=torch.float64, device=W.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=W.device)
    if ws is None:
        ws = torch.empty(max(256, math.ceil(In / 32) * R * 8), dtype=torch.uint8, device=W.device)
    _check(_lib.cprand_solve(In, R, _ptr(V), _ptr(W), dtype, _ptr(W_refine), _ptr(V_refine), _ptr(A_out),
                             _ptr(lambda_out), _ptr(info), _ptr(ws), ws.numel(), _stream()))
    return A_out, lambda_out, info


def cprand_fit_est(X, normX, A, lam, R, P_hat, seed, fit_out=None, ws=None):
    order = len(X.dims)
    if fit_out is None:
        fit_out = torch.empty(1, dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = workspace(X, R, 1, P_hat)
    arr = _ptr_array(A, order)
    _check(_lib.cprand_fit_est(C.byref(X.c()), _ptr(normX), arr, _ptr(lam), R, P_hat, C.c_uint64(seed),
                               _ptr(fit_out), _ptr(ws), ws.numel(), _stream()))
    return fit_out


def cprand_energy_proposals(X, normX, alpha=0.1, cdf_out=None, energy_out=None):
    """Slice-energy proposal tables of every mode (and the slice energies)."""
    dev = X.data.device
    order = len(X.dims)
    if cdf_out is None:
        cdf_out = [torch.empty(I + 1, dtype=torch.uint64, device=dev) for I in X.dims]
    if energy_out is None:
        energy_out = torch.empty(sum(X.dims), dtype=torch.float64, device=dev)
    ws = torch.empty(8 * sum(X.dims), dtype=torch.uint8, device=dev)
    _check(_lib.cprand_energy_proposals(C.byref(X.c()), _ptr(normX), alpha, _ptr_array(cdf_out, order),
                                        _ptr(energy_out), _ptr(ws), ws.numel(), _stream()))
    return cdf_out, energy_out


def cprand_fit_set_weighted(dims, P_hat, seed, cdf, beta, device="cuda"):
    order = len(dims)
    idx = torch.empty((P_hat, order), dtype=torch.int32, device=device)
    w = torch.empty(P_hat, dtype=torch.float64, device=device)
    _check(_lib.cprand_fit_set_weighted(order, (C.c_int64 * order)(*dims), P_hat, C.c_uint64(seed),
                                        _ptr_array(cdf, order), beta, _ptr(idx), _ptr(w), _stream()))
    return idx, w


def cprand_fit_est_weighted(X, normX, A, lam, R, P_hat, seed, cdf, beta, fit_out=None, ws=None):
    order = len(X.dims)
    if fit_out is None:
        fit_out = torch.empty(1, dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = torch.empty(int(_lib.cprand_fit_weighted_workspace_size(order, P_hat)), dtype=torch.uint8,
                         device=X.data.device)
    _check(_lib.cprand_fit_est_weighted(C.byref(X.c()), _ptr(normX), _ptr_array(A, order), _ptr(lam), R, P_hat,
                                        C.c_uint64(seed), _ptr_array(cdf, order), beta, _ptr(fit_out), _ptr(ws),
                                        ws.numel(), _stream()))
    return fit_out


def cprand_norm(X, out=None, ws=None):
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = torch.empty(4096 * 8, dtype=torch.uint8, device=X.data.device)
    _check(_lib.cprand_norm(C.byref(X.c()), _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def cprand_mix(X, seed, Xhat=None, signs=None, normX=None, ws=None):
    dev = X.data.device
    P = math.prod(X.dims)
    if Xhat is None:
        ct = torch.complex128 if X.dtype == F64 else torch.complex64
        Xhat = View(torch.empty(P, dtype=ct, device=dev), X.dims)
    if signs is None:
        signs = torch.empty(sum(X.dims), dtype=torch.int8, device=dev)
    if normX is None:
        normX = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = torch.empty(4096 * 8, dtype=torch.uint8, device=dev)
    _check(_lib.cprand_mix(C.byref(X.c()), C.c_uint64(seed), C.byref(Xhat.c()), _ptr(signs), _ptr(normX),
                           _ptr(ws), ws.numel(), _stream()))
    return Xhat, signs, normX


def cprand_mix_factor(A, signs, inverse=False, out=None):
    if not inverse:
        I, R = A.shape
        dtype = F64 if A.dtype == torch.float64 else F32
        if out is None:
            out = torch.empty((I, R), dtype=torch.complex128 if dtype == F64 else torch.complex64, device=A.device)
    else:
        I, R = A.shape
        dtype = F64 if A.dtype == torch.complex128 else F32
        if out is None:
            out = torch.empty((I, R), dtype=torch.float64 if dtype == F64 else torch.float32, device=A.device)
    _check(_lib.cprand_mix_factor(I, R, _ptr(A), dtype, _ptr(signs), _ptr(out), 1 if inverse else 0, _stream()))
    return out


def cprand_mix_dct(X, seed, Xhat=None, signs=None, normX=None, ws=None):
    dev = X.data.device
    P = math.prod(X.dims)
    if Xhat is None:
        Xhat = View(torch.empty(P, dtype=X.data.dtype, device=dev), X.dims)
    if signs is None:
        signs = torch.empty(sum(X.dims), dtype=torch.int8, device=dev)
    if normX is None:
        normX = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = torch.empty(4096 * 8, dtype=torch.uint8, device=dev)
    _check(_lib.cprand_mix_dct(C.byref(X.c()), C.c_uint64(seed), C.byref(Xhat.c()), _ptr(signs), _ptr(normX),
                               _ptr(ws), ws.numel(), _stream()))
    return Xhat, signs, normX


def cprand_mix_factor_dct(A, signs, inverse=False, out=None):
    I, R = A.shape
    dtype = F64 if A.dtype == torch.float64 else F32
    if out is None:
        out = torch.empty_like(A)
    _check(_lib.cprand_mix_factor_dct(I, R, _ptr(A), dtype, _ptr(signs), _ptr(out), 1 if inverse else 0, _stream()))
    return out


def full_workspace(X, R):
    return torch.empty(max(256, int(_lib.cprand_full_workspace_size(C.byref(X.c()), R))), dtype=torch.uint8,
                       device=X.data.device)


def cprand_mttkrp_full(X, n, A, R, W=None, ws=None):
    """W = X_(n) Z^(n) (FP64, I_n x R)."""
    order = len(X.dims)
    if W is None:
        W = torch.empty((X.dims[n], R), dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = full_workspace(X, R)
    arr = _ptr_array([None if m == n else A[m] for m in range(order)], order)
    _check(_lib.cprand_mttkrp_full(C.byref(X.c()), n, arr, R, _ptr(W), _ptr(ws), ws.numel(), _stream()))
    return W


def cprand_fit_exact(X, normX, A, lam, R, fit_out=None, ws=None):
    order = len(X.dims)
    if fit_out is None:
        fit_out = torch.empty(1, dtype=torch.float64, device=X.data.device)
    if ws is None:
        ws = full_workspace(X, R)
    arr = _ptr_array(A, order)
    _check(_lib.cprand_fit_exact(C.byref(X.c()), _ptr(normX), arr, _ptr(lam), R, _ptr(fit_out), _ptr(ws), ws.numel(),
                                 _stream()))
    return fit_out


def cprand_cpals(X, A, R, max_iters, tol=0.0):
    """Dense CP-ALS from A[1..N-1] (updated in place); returns lambda, the
    fit history and the status flags."""
    order = len(X.dims)
    lam = torch.empty(R, dtype=torch.float64, device=X.data.device)
    hist = (C.c_double * max_iters)()
    iters = C.c_int32(0)
    arr = _ptr_array(A, order)
    rc = _check(_lib.cprand_cpals(C.byref(X.c()), R, max_iters, tol, arr, _ptr(lam), hist, C.byref(iters), _stream()))
    return {"lambda": lam, "fit_history": list(hist[:iters.value]), "iters": iters.value, "flags": rc}


def cprand_mode_major_strides(dims, n, ld):
    order = len(dims)
    out = (C.c_int64 * order)()
    _check(_lib.cprand_mode_major_strides(order, (C.c_int64 * order)(*dims), n, ld, out))
    return tuple(out)


def cprand_layout_copy(X, n, Y):
    _check(_lib.cprand_layout_copy(C.byref(X.c()), n, C.byref(Y.c()), _stream()))
    return Y


def mode_major_copy(X, n, dtype=None, ld=None):
    """Allocate and fill a copy of X with mode n innermost (fibers contiguous)."""
    tdt = X.data.dtype if dtype is None else dtype
    esz = torch.empty(0, dtype=tdt).element_size()
    ve = 16 // esz
    ld = ld or ((X.dims[n] + ve - 1) // ve) * ve
    strides = cprand_mode_major_strides(X.dims, n, ld)
    P = math.prod(X.dims) // X.dims[n] * ld
    Y = View(torch.empty(P, dtype=tdt, device=X.data.device), X.dims, strides)
    return cprand_layout_copy(X, n, Y)


def cprand_mlp_param_count():
    return int(_lib.cprand_mlp_param_count())


def cprand_proposal(dims, n, R, A, kind, params=None, alpha=0.1, cdf_out=None, ws=None):
    """Integer proposal tables (list of device uint64 tensors, entry n None)."""
    order = len(dims)
    dev = A[(n + 1) % order].device
    if cdf_out is None:
        cdf_out = [None if m == n else torch.empty(dims[m] + 1, dtype=torch.uint64, device=dev)
                   for m in range(order)]
    cdims = (C.c_int64 * order)(*dims)
    if ws is None:
        ws = torch.empty(int(_lib.cprand_proposal_workspace_size(order, cdims, R)), dtype=torch.uint8, device=dev)
    _check(_lib.cprand_proposal(order, cdims, n, R, _ptr_array([None if m == n else A[m] for m in range(order)], order),
                                kind, _ptr(params), alpha, _ptr_array(cdf_out, order), _ptr(ws), ws.numel(),
                                _stream()))
    return cdf_out


def cprand_mlp_features(dims, n, R, A, with_targets=True, ws=None):
    """Feature rows (rows x 4) and exact-marginal targets for mode step n."""
    order = len(dims)
    dev = A[(n + 1) % order].device
    rows = sum(d for m, d in enumerate(dims) if m != n)
    X = torch.empty((rows, 4), dtype=torch.float32, device=dev)
    t = torch.empty(rows, dtype=torch.float32, device=dev) if with_targets else None
    cdims = (C.c_int64 * order)(*dims)
    if ws is None:
        ws = torch.empty(int(_lib.cprand_proposal_workspace_size(order, cdims, R)), dtype=torch.uint8, device=dev)
    _check(_lib.cprand_mlp_features(order, cdims, n, R, _ptr_array([None if m == n else A[m] for m in range(order)],
                                                                    order),
                                    _ptr(X), _ptr(t), _ptr(ws), ws.numel(), _stream()))
    return X, t


def cprand_mlp_forward(params, X):
    z = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(_lib.cprand_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(z), _stream()))
    return z


def cprand_mlp_grad(params, X, t, group_off, grad=None, loss=None, ws=None):
    rows, ng = X.shape[0], group_off.numel() - 1
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
    if ws is None:
        ws = torch.empty(int(_lib.cprand_mlp_workspace_size(rows, ng)), dtype=torch.uint8, device=X.device)
    _check(_lib.cprand_mlp_grad(_ptr(params), _ptr(X), _ptr(t), _ptr(group_off), ng, rows, _ptr(grad), _ptr(loss),
                                _ptr(ws), ws.numel(), _stream()))
    return grad, loss


def cprand_mlp_adam(params, grad, m, v, step, lr=1e-3):
    _check(_lib.cprand_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, _stream()))
    return params


def cprand_mlp_train(params, X, t, group_off, epochs, lr=1e-3):
    hist = (C.c_double * epochs)()
    _check(_lib.cprand_mlp_train(_ptr(params), _ptr(X), _ptr(t), _ptr(group_off), group_off.numel() - 1, X.shape[0],
                                 epochs, lr, hist, _stream()))
    return [hist[i] for i in range(epochs)]


def make_opts(R, S, P_hat=2 ** 14, max_iters=50, seed=0, tol=0.0, fit_target=2.0, patience=0,
              mix=MIX_NONE, precision=PREC_NATIVE, proposal=PROPOSAL_UNIFORM, layout=0, use_graph=1,
              alpha=0.1, proposal_cdf=None, mlp_params=None, refine_every=0, fit_beta=0.0, fit_alpha=0.1):
    o = _abi.cprand_opts()
    o.R, o.S, o.P_hat, o.max_iters = R, S, P_hat, max_iters
    o.seed = seed
    o.tol, o.fit_target, o.patience = tol, (2.0 if fit_target is None else fit_target), patience
    o.mix, o.precision, o.proposal, o.layout, o.use_graph = mix, precision, proposal, layout, use_graph
    o.alpha = alpha
    o.refine_every = refine_every
    o.fit_beta, o.fit_alpha = fit_beta, fit_alpha
    keep = []
    if proposal_cdf is not None:
        arr = (C.c_void_p * len(proposal_cdf))(*[c.data_ptr() for c in proposal_cdf])
        o.proposal_cdf = C.cast(arr, C.POINTER(C.c_void_p))
        keep.append(arr)
    if mlp_params is not None:
        o.mlp_params = mlp_params.data_ptr()
    o._keep = keep
    return o


class Plan:
    """cprand_plan_create / cprand_plan_run / cprand_plan_destroy."""

    def __init__(self, X, opts):
        self.opts = opts
        self.X = X
        h = C.c_void_p()
        _check(_lib.cprand_plan_create(C.byref(X.c()), C.byref(opts), C.byref(h)))
        self.h = h

    def run(self, X, A, lam=None):
        order = len(X.dims)
        if lam is None:
            lam = torch.empty(self.opts.R, dtype=torch.float64, device=X.data.device)
        hist = (C.c_double * self.opts.max_iters)()
        props = (C.c_int32 * self.opts.max_iters)()
        rep = _abi.cprand_report()
        rep.fit_history = hist
        rep.proposal_history = props
        rc = _check(_lib.cprand_plan_run(self.h, C.byref(X.c()), _ptr_array(A, order), _ptr(lam), C.byref(rep),
                                         _stream()))
        return {"status": rc, "lambda": lam, "iters": rep.iters, "flags": rep.flags, "fit_est": rep.fit_est,
                "setup_ms": rep.setup_ms, "loop_ms": rep.loop_ms, "norm_ms": rep.norm_ms,
                "mix_ms": [rep.mix_ms[i] for i in range(order)],
                "layout_ms": [rep.layout_ms[i] for i in range(order)], "fused": rep.fused,
                "refined_from": rep.refined_from,
                "fit_history": [hist[i] for i in range(rep.iters)],
                "proposal_history": [props[i] for i in range(rep.iters)]}

    def close(self):
        if self.h:
            _lib.cprand_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cprand_plan_create(X, opts):
    return Plan(X, opts)


def cprand_als(X, A, opts):
    """Whole decomposition; A: list of (I_m, R) device tensors (A[1:] = init),
    overwritten with the result.  Returns the run record (with lambda)."""
    p = Plan(X, opts)
    try:
        return p.run(X, A)
    finally:
        p.close()
