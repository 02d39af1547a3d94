"""ctypes binding of libtp.so: argument marshalling only (names follow include/tp.h)."""
import ctypes as C
import os

import numpy as np

TP_OK, TP_EINVAL, TP_ENOMEM, TP_ENOCONV, TP_ERANK, TP_EHIP, TP_EINDEF = range(7)
TP_FP64, TP_MIXED = 0, 1
TP_SYM_FIT, TP_SYM_SINC = 0, 1
TP_STOP_ERROR, TP_STOP_RESIDUAL = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def library_path():
    return os.path.join(_HERE, "libtp.so")


class TPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tp status %d: %s" % (status, msg))
        self.status = status


class tp_tensor(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32 * 3), ("cap", C.c_int32), ("prec", C.c_int32),
                ("rank", C.c_int32 * 3), ("core", C.c_void_p), ("factor", C.c_void_p * 3)]


class tp_cp(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32 * 3), ("rank", C.c_int32),
                ("weight", C.c_void_p), ("factor", C.c_void_p * 3)]


class tp_sketch(C.Structure):
    _fields_ = [("q", C.c_int32), ("omega", C.c_void_p * 3)]


class tp_symbol_desc(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32 * 3), ("alpha", C.c_double), ("c_neg", C.c_double),
                ("c_pos", C.c_double), ("method", C.c_int32), ("op_terms", C.c_int32),
                ("pre_terms", C.c_int32), ("sinc_kl", C.c_int32), ("sinc_kr", C.c_int32),
                ("sinc_h", C.c_double), ("prec", C.c_int32), ("c0", C.c_double), ("beta", C.c_double),
                ("pre_rank", C.c_int32), ("directional", C.c_int32)]


class tp_pcg_opts(C.Structure):
    _fields_ = [("tau", C.c_double), ("kmax", C.c_int32), ("trunc_tol", C.c_double), ("cap", C.c_int32),
                ("true_residual", C.c_int32), ("stop_rule", C.c_int32),
                ("recursive_residual", C.c_int32), ("spectral_domain", C.c_int32), ("warm_start", C.c_int32)]


class tp_pcg_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rank", C.c_int32 * 3),
                ("rel_res", C.c_double), ("true_rel_res", C.c_double), ("op_applies", C.c_double),
                ("err_est", C.c_double)]


P = C.c_void_p
_SIGS = {
    "tp_version": ([], C.c_int),
    "tp_last_error": ([], C.c_char_p),
    "tp_create": ([C.c_int, P, C.c_size_t, C.POINTER(P)], C.c_int),
    "tp_destroy": ([P], C.c_int),
    "tp_symbol_build": ([P, C.POINTER(tp_symbol_desc), C.POINTER(P), C.POINTER(P), C.POINTER(C.c_double)], C.c_int),
    "tp_symbol_free": ([P], C.c_int),
    "tp_state_symbol_build": ([P, C.POINTER(tp_symbol_desc), C.POINTER(P), C.POINTER(C.c_double)], C.c_int),
    "tp_symbol_info": ([P, C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
    "tp_symbol_eval": ([P, P, C.c_int32, P, P], C.c_int),
    "tp_from_cp": ([P, C.POINTER(tp_cp), C.POINTER(tp_tensor), C.c_double], C.c_int),
    "tp_apply": ([P, P, C.POINTER(tp_tensor), C.POINTER(tp_tensor), C.c_double, C.c_int32,
                  C.POINTER(tp_sketch)], C.c_int),
    "tp_truncate": ([P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.POINTER(tp_tensor)),
                     C.POINTER(tp_tensor), C.c_double, C.c_int32], C.c_int),
    "tp_inner": ([P, C.POINTER(tp_tensor), C.POINTER(tp_tensor), C.POINTER(C.c_double)], C.c_int),
    "tp_inner_noalloc": ([P, C.POINTER(tp_tensor), C.POINTER(tp_tensor), P], C.c_int),
    "tp_inner_sym": ([P, C.POINTER(tp_tensor), P, C.POINTER(tp_tensor), C.POINTER(C.c_double)], C.c_int),
    "tp_apply_sum": ([P, C.c_int32, C.POINTER(P), C.POINTER(C.POINTER(tp_tensor)), C.POINTER(C.c_double),
                      C.POINTER(tp_tensor), C.c_double, C.c_int32, C.POINTER(tp_sketch)], C.c_int),
    "tp_eval_grid": ([P, C.POINTER(tp_tensor), C.POINTER(P), C.POINTER(C.c_int32), P], C.c_int),
    "tp_workspace_query": ([C.POINTER(tp_symbol_desc), C.POINTER(tp_pcg_opts), C.c_int32, C.c_int32,
                            C.POINTER(C.c_size_t)], C.c_int),
    "tp_workspace_peak": ([P, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "tp_pcg_solve": ([P, P, P, C.POINTER(tp_cp), C.POINTER(tp_tensor), C.POINTER(tp_pcg_opts),
                      C.POINTER(tp_sketch), C.POINTER(tp_pcg_info)], C.c_int),
    "tp_dst": ([P, C.c_int32, C.c_int32, C.c_int32, P, P], C.c_int),
    "tp_pcg_solve_batched": ([P, C.c_int32, C.POINTER(tp_symbol_desc), C.POINTER(tp_cp), C.POINTER(tp_tensor),
                              C.POINTER(tp_pcg_opts), C.POINTER(tp_sketch), C.POINTER(tp_pcg_info), C.c_int32,
                              C.c_size_t], C.c_int),
    "tp_syev": ([P, C.c_int32, C.c_int32, P, P, P], C.c_int),
    "tp_lambda": ([P, C.c_int32, P], C.c_int),
    "tp_gram_eig": ([P, C.c_int32, C.c_int32, P, P, P, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)],
                    C.c_int),
    "tp_profile": ([P, C.c_int32], C.c_int),
    "tp_gemm_mode": ([C.c_int32], C.c_int),
    "tp_profile_read": ([P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                         C.POINTER(C.c_double)], C.c_int),
}

PROF_CLASSES = ["gemm_f64", "gemm_f32", "gemm_f32_f64", "gemm_f64_f32", "dst_f64", "dst_f32", "syev", "chol",
                "psd_eig", "ns_isqrt", "gemm_reduce", "psd_tri", "gemm_f32_split64"]


def load_library():
    """Load libtp.so (raises OSError when it has not been built)."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise OSError("libtp.so not built: run __graft_entry__.build() (expected at %s)" % path)
        lib = C.CDLL(path)
        for name, (args, res) in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _LIB = lib
    return _LIB


def exported_symbols():
    return list(_SIGS)


def _check(status, allow=()):
    if status != TP_OK and status not in allow:
        msg = load_library().tp_last_error().decode(errors="replace")
        raise TPError(status, msg)
    return status


def _torch():
    import torch
    return torch


def _dtype(prec):
    t = _torch()
    return t.float64 if prec == TP_FP64 else t.float32


class Context:
    """tp_ctx on a CUDA/HIP device, ordering work on torch's current stream."""

    def __init__(self, device=0, workspace_bytes=0):
        t = _torch()
        self.lib = load_library()
        self.device = device
        t.cuda.set_device(device)
        self.stream = t.cuda.current_stream(device)
        h = P()
        _check(self.lib.tp_create(device, P(self.stream.cuda_stream), workspace_bytes, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- kernel-level entry points
    def dst(self, x, out=None):
        t = _torch()
        prec = TP_FP64 if x.dtype == t.float64 else TP_MIXED
        x = x.contiguous()
        n, cols = (x.shape[0], 1) if x.dim() == 1 else (x.shape[0], x.shape[1])
        # column-major columns of length n: a torch (cols, n) tensor is that layout
        xc = x.t().contiguous() if x.dim() == 2 else x
        out_t = t.empty_like(xc) if out is None else out
        _check(self.lib.tp_dst(self.h, n, cols, prec, P(xc.data_ptr()), P(out_t.data_ptr())))
        return out_t.t() if x.dim() == 2 else out_t

    def gram_eig(self, a, cut=0.0):
        """a: (count, K, K) float64 CUDA tensor of positive semidefinite matrices -> (w, v, ranks, rest):
        w (count, K) descending, v (count, K, K) with v[b][:, i] the i-th eigenvector (column-major
        rows of the torch tensor are columns), ranks and rest as lists."""
        t = _torch()
        a = a.contiguous()
        cnt, K, _ = a.shape
        w = t.empty((cnt, K), dtype=t.float64, device=a.device)
        v = t.empty((cnt, K, K), dtype=t.float64, device=a.device)
        rk = (C.c_int32 * cnt)()
        rs = (C.c_double * cnt)()
        _check(self.lib.tp_gram_eig(self.h, K, cnt, P(a.data_ptr()), P(w.data_ptr()), P(v.data_ptr()), cut, rk, rs))
        return w, v, list(rk), list(rs)

    def syev(self, a):
        """a: (count, K, K) float64 CUDA tensor of symmetric matrices."""
        t = _torch()
        a = a.contiguous()
        cnt, K, _ = a.shape
        w = t.empty((cnt, K), dtype=t.float64, device=a.device)
        v = t.empty((cnt, K, K), dtype=t.float64, device=a.device)
        _check(self.lib.tp_syev(self.h, K, cnt, P(a.data_ptr()), P(w.data_ptr()), P(v.data_ptr())))
        # v is column-major per matrix: v[b] stored as (K x K) col-major -> transpose view
        return w, v.transpose(1, 2)

    def lam(self, n):
        t = _torch()
        out = t.empty(n, dtype=t.float64, device="cuda")
        _check(self.lib.tp_lambda(self.h, n, P(out.data_ptr())))
        return out

    # ---- measurement
    def gemm_mode(self, mfma=True):
        """tp_gemm_mode: True / 1 matrix cores (default), False / 0 FMA tiles, 2 split-BF16 products
        for the FP32 contractions."""
        _check(self.lib.tp_gemm_mode(int(mfma)))

    def profile(self, enable=True):
        _check(self.lib.tp_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        out = {}
        for i, name in enumerate(PROF_CLASSES):
            v = [C.c_double() for _ in range(4)]
            _check(self.lib.tp_profile_read(self.h, i, *[C.byref(x) for x in v]))
            out[name] = {"ms": v[0].value, "launches": v[1].value, "flops": v[2].value, "bytes": v[3].value}
        return out

    # ---- workspace
    def workspace_peak(self, reset=False):
        v = C.c_size_t()
        _check(self.lib.tp_workspace_peak(self.h, 1 if reset else 0, C.byref(v)))
        return v.value

    # ---- symbols
    def symbol_build(self, d, n, alpha, c_neg, c_pos, prec=TP_FP64, method=TP_SYM_FIT, op_terms=0,
                     pre_terms=0, sinc_kl=0, sinc_kr=0, sinc_h=0.0, c0=0.0, beta=0.0, pre_rank=0,
                     directional=False, allow_indefinite=False):
        """Operator and preconditioner symbols and their measured errors.  A preconditioner that is
        not positive on its checked points (TP_EINDEF) raises unless allow_indefinite; then the
        symbols are returned and `indefinite` is set on the preconditioner."""
        desc = tp_symbol_desc()
        desc.d = d
        ns = mode_sizes(d, n)
        for m in range(3):
            desc.n[m] = ns[m] if m < d else 0
        desc.alpha, desc.c_neg, desc.c_pos = alpha, c_neg, c_pos
        desc.c0, desc.beta, desc.pre_rank = c0, beta, pre_rank
        desc.directional = 1 if directional else 0
        desc.method, desc.op_terms, desc.pre_terms = method, op_terms, pre_terms
        desc.sinc_kl, desc.sinc_kr, desc.sinc_h = sinc_kl, sinc_kr, sinc_h
        desc.prec = prec
        op, pre = P(), P()
        err = (C.c_double * 2)()
        st = self.lib.tp_symbol_build(self.h, C.byref(desc), C.byref(op), C.byref(pre), err)
        if st == TP_EINDEF:
            so, sp = Symbol(self, op, d, prec), Symbol(self, pre, d, prec)
            sp.indefinite = True
            if allow_indefinite:
                return so, sp, (err[0], err[1])
            msg = self.lib.tp_last_error().decode(errors="replace")
            so.free()
            sp.free()
            raise TPError(st, msg)
        _check(st)
        return Symbol(self, op, d, prec), Symbol(self, pre, d, prec), (err[0], err[1])

    def state_symbol_build(self, d, n, alpha, beta, prec=TP_FP64, terms=0, directional=False):
        desc = tp_symbol_desc()
        desc.d = d
        ns = mode_sizes(d, n)
        for m in range(3):
            desc.n[m] = ns[m] if m < d else 0
        desc.alpha, desc.c_neg, desc.c_pos = alpha, beta, 0.0
        desc.op_terms, desc.prec = terms, prec
        desc.directional = 1 if directional else 0
        h = P()
        err = C.c_double()
        _check(self.lib.tp_state_symbol_build(self.h, C.byref(desc), C.byref(h), C.byref(err)))
        return Symbol(self, h, d, prec), err.value

    # ---- tensors
    def from_cp(self, weights, factors, out, tol=0.0, allow_erank=False):
        keep, cp = cp_struct(weights, factors)
        st = _check(self.lib.tp_from_cp(self.h, C.byref(cp), C.byref(out.s), tol),
                    allow=(TP_ERANK,) if allow_erank else ())
        out._sync_ranks()
        return st

    def apply(self, sym, x, y, tol, cap, sketch, allow_erank=False):
        sk, keep = sketch_struct(sketch)
        st = _check(self.lib.tp_apply(self.h, sym.h, C.byref(x.s), C.byref(y.s), tol, cap, C.byref(sk)),
                    allow=(TP_ERANK,) if allow_erank else ())
        y._sync_ranks()
        return st

    def truncate(self, coefs, xs, y, tol, cap, allow_erank=False):
        n = len(xs)
        cf = (C.c_double * n)(*coefs)
        arr = (C.POINTER(tp_tensor) * n)(*[C.pointer(x.s) for x in xs])
        st = _check(self.lib.tp_truncate(self.h, n, cf, arr, C.byref(y.s), tol, cap),
                    allow=(TP_ERANK,) if allow_erank else ())
        y._sync_ranks()
        return st

    def apply_sum(self, syms, xs, coefs, y, tol, cap, sketch, allow_erank=False):
        n = len(xs)
        sk, keep = sketch_struct(sketch)
        sa = (P * n)(*[s.h if s is not None else None for s in syms])
        arr = (C.POINTER(tp_tensor) * n)(*[C.pointer(x.s) for x in xs])
        cf = (C.c_double * n)(*coefs)
        st = _check(self.lib.tp_apply_sum(self.h, n, sa, arr, cf, C.byref(y.s), tol, cap, C.byref(sk)),
                    allow=(TP_ERANK,) if allow_erank else ())
        y._sync_ranks()
        return st

    def inner_sym(self, x, sym, y):
        out = C.c_double()
        _check(self.lib.tp_inner_sym(self.h, C.byref(x.s), sym.h, C.byref(y.s), C.byref(out)))
        return out.value

    def inner(self, x, y):
        out = C.c_double()
        _check(self.lib.tp_inner(self.h, C.byref(x.s), C.byref(y.s), C.byref(out)))
        return out.value

    def inner_noalloc(self, x, y, out=None):
        """tp_inner_noalloc: <x, y> into a device double (a 1-element float64 CUDA tensor, returned)."""
        t = _torch()
        if out is None:
            out = t.empty(1, dtype=t.float64, device="cuda")
        _check(self.lib.tp_inner_noalloc(self.h, C.byref(x.s), C.byref(y.s), P(out.data_ptr())))
        return out

    def eval_grid(self, x, rows):
        t = _torch()
        rs = [t.as_tensor(np.asarray(r, dtype=np.int32), device="cuda") for r in rows]
        m = (C.c_int32 * 3)(*([len(r) for r in rows] + [1] * (3 - len(rows))))
        ptrs = (P * 3)(*([P(r.data_ptr()) for r in rs] + [None] * (3 - len(rs))))
        out = t.empty(int(np.prod([len(r) for r in rows])), dtype=t.float64, device="cuda")
        _check(self.lib.tp_eval_grid(self.h, C.byref(x.s), ptrs, m, P(out.data_ptr())))
        # column-major (m0, m1, m2) -> numpy C-order array indexed [i0, i1, i2]
        return out.cpu().numpy().reshape([len(r) for r in rows][::-1]).transpose(
            list(range(len(rows)))[::-1])

    def pcg_solve(self, op, pre, weights, factors, x, tau, kmax, trunc_tol, cap, sketch, true_residual=False,
                  allow=(TP_ERANK, TP_ENOCONV), stop_rule=0, recursive_residual=False, spectral_domain=False,
                  warm_start=False):
        if isinstance(weights, Rhs):  # already on the device
            keep, cp = weights.keep, weights.cp
        else:
            keep, cp = cp_struct(weights, factors)
        sk, keep2 = sketch_struct(sketch)
        o = tp_pcg_opts(tau, kmax, trunc_tol, cap, 1 if true_residual else 0, stop_rule,
                        1 if recursive_residual else 0, 1 if spectral_domain else 0, 1 if warm_start else 0)
        info = tp_pcg_info()
        st = _check(self.lib.tp_pcg_solve(self.h, op.h, pre.h, C.byref(cp), C.byref(x.s), C.byref(o),
                                          C.byref(sk), C.byref(info)), allow=allow)
        x._sync_ranks()
        return st, {"iters": info.iters, "status": info.status, "rank": list(info.rank)[:x.d],
                    "rel_res": info.rel_res, "true_rel_res": info.true_rel_res,
                    "applies": info.op_applies, "err_est": info.err_est}


def _desc(d, n, alpha, c_neg, c_pos, prec, op_terms, pre_terms, **kw):
    """tp_symbol_desc; kw sets further fields by name (method, sinc_kl, c0, beta, pre_rank, ...)."""
    desc = tp_symbol_desc()
    desc.d = d
    ns = mode_sizes(d, n)
    for m in range(3):
        desc.n[m] = ns[m] if m < d else 0
    desc.alpha, desc.c_neg, desc.c_pos = alpha, c_neg, c_pos
    desc.method, desc.op_terms, desc.pre_terms = TP_SYM_FIT, op_terms, pre_terms
    desc.prec = prec
    for k, v in kw.items():
        setattr(desc, k, v)
    return desc


_DESC_KEYS = ("method", "sinc_kl", "sinc_kr", "sinc_h", "pre_rank", "directional")


def workspace_query(d, n, alpha, settings, rhs_rank, c_neg=1.0, c_pos=1e-2, **desc_kw):
    """tp_workspace_query for a symbol descriptor and PCG settings (prec, eps, tau, cap, q, op_terms,
    pre_terms): the estimated workspace bytes of one symbol build and solve."""
    desc = _desc(d, n, alpha, c_neg, c_pos, settings["prec"], settings["op_terms"], settings["pre_terms"])
    for k, v in desc_kw.items():
        setattr(desc, k, v)
    o = tp_pcg_opts(settings["tau"], 100, settings["eps"], settings["cap"], 0, 0, 0, 0, 0)
    v = C.c_size_t()
    _check(load_library().tp_workspace_query(C.byref(desc), C.byref(o), settings["q"], rhs_rank, C.byref(v)))
    return v.value


def batch_solve(ctx, problems, settings, sketches, streams=8, workspace_per_stream=0, rhs=None):
    """Solve independent problems concurrently (tp_pcg_solve_batched).  settings(p) -> dict with
    prec, eps, tau, cap, op_terms, pre_terms (and optionally q); sketches[(n, q)] or sketches[n] -> device
    sketch tensors for grid n; rhs: optional list of `Rhs` (the problems' right-hand sides already on
    the device), else they are copied here."""
    cnt = len(problems)
    descs = (tp_symbol_desc * cnt)()
    cps = (tp_cp * cnt)()
    tens = (tp_tensor * cnt)()
    opts = (tp_pcg_opts * cnt)()
    sks = (tp_sketch * cnt)()
    infos = (tp_pcg_info * cnt)()
    keep, outs = [], []
    for i, p in enumerate(problems):
        s = settings(p)
        extra = {k: s[k] for k in _DESC_KEYS if k in s}
        descs[i] = _desc(p.d, p.n, p.alpha, p.c_neg, p.c_pos, s["prec"], s["op_terms"], s["pre_terms"],
                         c0=getattr(p, "c0", 0.0) or 0.0, beta=getattr(p, "beta", None) or 0.0, **extra)
        k, cp = (rhs[i].keep, rhs[i].cp) if rhs is not None else cp_struct(p.weights, p.factors)
        keep.append(k)
        cps[i] = cp
        X = Tensor(p.d, p.n, s["cap"], s["prec"])
        outs.append(X)
        tens[i] = X.s
        opts[i] = tp_pcg_opts(s["tau"], s.get("kmax", 100), s["eps"], s["cap"], 0, s.get("stop_rule", 0),
                              1 if s.get("recursive_residual") else 0, 1 if s.get("spectral") else 0, 0)
        key = (p.n, s["q"]) if "q" in s else None
        sk, k2 = sketch_struct(sketches[key] if key in sketches else sketches[p.n])
        sks[i] = sk
    _check(ctx.lib.tp_pcg_solve_batched(ctx.h, cnt, descs, cps, tens, opts, sks, infos, streams,
                                         workspace_per_stream))
    res = []
    for i, X in enumerate(outs):
        X.s = tens[i]
        X._sync_ranks()
        res.append({"iters": infos[i].iters, "status": infos[i].status, "rank": list(infos[i].rank)[:X.d],
                    "err_est": infos[i].err_est})
    return outs, res


class Symbol:
    def __init__(self, ctx, h, d, prec):
        self.ctx, self.h, self.d, self.prec = ctx, h, d, prec
        self.indefinite = False

    def info(self):
        r, e = C.c_int32(), C.c_double()
        _check(self.ctx.lib.tp_symbol_info(self.h, C.byref(r), C.byref(e)))
        return r.value, e.value

    def eval(self, idx):
        """idx: (count, d) int array of 0-based multi-indices -> values (numpy)."""
        t = _torch()
        it = t.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device="cuda")
        out = t.empty(it.shape[0], dtype=t.float64, device="cuda")
        _check(self.ctx.lib.tp_symbol_eval(self.ctx.h, self.h, it.shape[0], P(it.data_ptr()), P(out.data_ptr())))
        return out.cpu().numpy()

    def free(self):
        if self.h:
            self.ctx.lib.tp_symbol_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mode_sizes(d, n):
    """Grid sizes per mode from an int (every mode) or a sequence of d ints."""
    ns = [int(v) for v in n] if hasattr(n, "__len__") else [int(n)] * d
    if len(ns) != d:
        raise ValueError("need %d mode sizes, got %s" % (d, n))
    return ns


class Tensor:
    """Tucker tensor in torch-owned device memory (core cap^d, factors n_l x cap column-major).
    n: one grid size for every mode or one per mode."""

    def __init__(self, d, n, cap, prec=TP_FP64, device="cuda"):
        t = _torch()
        self.ns = mode_sizes(d, n)
        self.d, self.n, self.cap, self.prec = d, n, cap, prec
        dt = _dtype(prec)
        self.core = t.zeros(cap ** d, dtype=dt, device=device)
        self.factors = [t.zeros(cap * self.ns[m], dtype=dt, device=device) for m in range(d)]
        s = tp_tensor()
        s.d, s.cap, s.prec = d, cap, prec
        for m in range(3):
            s.n[m] = self.ns[m] if m < d else 0
            s.rank[m] = 0
        s.core = self.core.data_ptr()
        for m in range(d):
            s.factor[m] = self.factors[m].data_ptr()
        self.s = s
        self.rank = [0] * d

    def _sync_ranks(self):
        self.rank = [self.s.rank[m] for m in range(self.d)]

    def numpy_parts(self):
        """(core, [factors]) as float64 numpy arrays with the current ranks."""
        r = self.rank
        core = self.core[: int(np.prod(r))].double().cpu().numpy().reshape(r[::-1]).transpose(
            list(range(self.d))[::-1])
        fs = [self.factors[m][: self.ns[m] * r[m]].double().cpu().numpy().reshape(r[m], self.ns[m]).T
              for m in range(self.d)]
        return core, fs


class Rhs:
    """A canonical right-hand side (weights, n x R factors) copied to the device once, for solves
    that take their input from device memory."""

    def __init__(self, weights, factors):
        self.keep, self.cp = cp_struct(weights, factors)


def cp_struct(weights, factors):
    """Device copies of a canonical tensor (float64) and its tp_cp struct."""
    t = _torch()
    w = t.as_tensor(np.asarray(weights, dtype=np.float64), device="cuda")
    fs = [t.as_tensor(np.asfortranarray(np.asarray(f, dtype=np.float64)).T.copy(), device="cuda")
          for f in factors]   # (R, n) C-order == (n, R) column-major
    cp = tp_cp()
    cp.d = len(factors)
    for m in range(3):
        cp.n[m] = factors[m].shape[0] if m < cp.d else 0
    cp.rank = len(weights)
    cp.weight = w.data_ptr()
    for m in range(cp.d):
        cp.factor[m] = fs[m].data_ptr()
    return (w, fs), cp


def sketch_struct(sketch):
    """sketch: list of d torch float64 CUDA tensors of shape (q, n) (== n x q column-major)."""
    sk = tp_sketch()
    sk.q = sketch[0].shape[0]
    for m, o in enumerate(sketch):
        sk.omega[m] = o.data_ptr()
    return sk, sketch


def sketch_tensors(omegas):
    """numpy (n, q) Gaussian matrices -> device tensors in the layout the library reads."""
    t = _torch()
    return [t.as_tensor(np.ascontiguousarray(np.asarray(o, dtype=np.float64).T), device="cuda") for o in omegas]
