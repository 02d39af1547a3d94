"""Host-side behaviour of the C ABI that needs no device: argument checks of every entry point, the
workspace estimate (tp_workspace_query takes no context), and the absence of any host fallback in
the package.  Each library call here returns before any HIP call is made, so the tests run on a
machine without a GPU."""
import ctypes as C
import os

import pytest

from paper_1809_01971_amd import _tp

pytestmark = pytest.mark.skipif(not os.path.exists(_tp.library_path()), reason="libtp.so not built")

NULL = None


def _lib():
    return _tp.load_library()


def _err():
    return _lib().tp_last_error().decode(errors="replace")


def test_null_arguments_rejected_by_every_entry_point():
    """Every entry point that takes a context or an output pointer rejects NULL with TP_EINVAL and
    leaves a message; the two release calls accept NULL (nothing to release)."""
    lib = _lib()
    t = _tp.tp_tensor()
    cp = _tp.tp_cp()
    sk = _tp.tp_sketch()
    desc = _tp._desc(3, 127, 0.5, 1.0, 1e-2, _tp.TP_MIXED, 28, 12)
    opts = _tp.tp_pcg_opts(1e-5, 10, 1e-5, 50, 0, 0, 0, 0, 0)
    info = _tp.tp_pcg_info()
    d = C.c_double()
    h = C.c_void_p()
    sz = C.c_size_t()
    calls = {
        "tp_create": lambda: lib.tp_create(0, NULL, 0, NULL),
        "tp_symbol_build": lambda: lib.tp_symbol_build(NULL, C.byref(desc), C.byref(h), C.byref(h), NULL),
        "tp_state_symbol_build": lambda: lib.tp_state_symbol_build(NULL, C.byref(desc), C.byref(h), NULL),
        "tp_symbol_info": lambda: lib.tp_symbol_info(NULL, NULL, NULL),
        "tp_symbol_eval": lambda: lib.tp_symbol_eval(NULL, NULL, 0, NULL, NULL),
        "tp_from_cp": lambda: lib.tp_from_cp(NULL, C.byref(cp), C.byref(t), 1e-6),
        "tp_apply": lambda: lib.tp_apply(NULL, NULL, C.byref(t), C.byref(t), 1e-6, 8, C.byref(sk)),
        "tp_apply_sum": lambda: lib.tp_apply_sum(NULL, 1, NULL, NULL, NULL, C.byref(t), 1e-6, 8, C.byref(sk)),
        "tp_inner_sym": lambda: lib.tp_inner_sym(NULL, C.byref(t), NULL, C.byref(t), C.byref(d)),
        "tp_truncate": lambda: lib.tp_truncate(NULL, 1, NULL, NULL, C.byref(t), 1e-6, 8),
        "tp_inner": lambda: lib.tp_inner(NULL, C.byref(t), C.byref(t), C.byref(d)),
        "tp_inner_noalloc": lambda: lib.tp_inner_noalloc(NULL, C.byref(t), C.byref(t), NULL),
        "tp_eval_grid": lambda: lib.tp_eval_grid(NULL, C.byref(t), NULL, NULL, NULL),
        "tp_pcg_solve": lambda: lib.tp_pcg_solve(NULL, NULL, NULL, C.byref(cp), C.byref(t), C.byref(opts),
                                                 C.byref(sk), C.byref(info)),
        "tp_pcg_solve_batched": lambda: lib.tp_pcg_solve_batched(NULL, 1, C.byref(desc), C.byref(cp), C.byref(t),
                                                                 C.byref(opts), C.byref(sk), C.byref(info), 1, 0),
        "tp_workspace_query": lambda: lib.tp_workspace_query(C.byref(desc), C.byref(opts), 16, 1, NULL),
        "tp_workspace_peak": lambda: lib.tp_workspace_peak(NULL, 0, C.byref(sz)),
        "tp_dst": lambda: lib.tp_dst(NULL, 127, 1, _tp.TP_FP64, NULL, NULL),
        "tp_syev": lambda: lib.tp_syev(NULL, 8, 1, NULL, NULL, NULL),
        "tp_gram_eig": lambda: lib.tp_gram_eig(NULL, 8, 1, NULL, NULL, NULL, 0.0, NULL, NULL),
        "tp_lambda": lambda: lib.tp_lambda(NULL, 127, NULL),
        "tp_profile": lambda: lib.tp_profile(NULL, 1),
        "tp_profile_read": lambda: lib.tp_profile_read(NULL, 0, NULL, NULL, NULL, NULL),
    }
    for name, call in calls.items():
        st = call()
        assert st == _tp.TP_EINVAL, (name, st)
        assert _err(), name
    assert lib.tp_destroy(NULL) == _tp.TP_OK
    assert lib.tp_symbol_free(NULL) == _tp.TP_OK
    # every declared entry point is either checked above or takes no pointer argument
    untested = set(_tp.exported_symbols()) - set(calls) - {"tp_destroy", "tp_symbol_free"}
    assert untested == {"tp_version", "tp_last_error", "tp_gemm_mode"}, untested


def test_the_error_message_names_the_failed_check():
    lib = _lib()
    opts = _tp.tp_pcg_opts(1e-5, 10, 1e-5, 50, 0, 0, 0, 0, 0)
    desc = _tp._desc(3, 127, 0.5, 1.0, 1e-2, _tp.TP_MIXED, 28, 12)
    desc.d = 4
    sz = C.c_size_t()
    assert lib.tp_workspace_query(C.byref(desc), C.byref(opts), 16, 1, C.byref(sz)) == _tp.TP_EINVAL
    assert "d=4" in _err()
    # a later failure replaces the message
    assert lib.tp_pcg_solve_batched(NULL, 1, NULL, NULL, NULL, NULL, NULL, NULL, 1, 0) == _tp.TP_EINVAL
    assert "NULL" in _err()


def _query(d=3, n=2047, prec=_tp.TP_MIXED, cap=50, q=80, rb=1, **kw):
    desc = _tp._desc(d, n, 0.5, 1.0, 1e-2, prec, kw.pop("op_terms", 28), kw.pop("pre_terms", 12), **kw)
    opts = _tp.tp_pcg_opts(1e-5, 10, 1e-5, cap, 0, 0, 0, 0, 0)
    sz = C.c_size_t()
    st = _lib().tp_workspace_query(C.byref(desc), C.byref(opts), q, rb, C.byref(sz))
    return st, sz.value


def test_workspace_query_is_monotone_in_every_size():
    """The estimate needs no context and grows with the grid, the rank cap, the sketch width, the
    right-hand side's rank and the number of symbol terms; FP64 tensors need more than FP32 ones."""
    st, base = _query()
    assert st == _tp.TP_OK and base > (64 << 20)
    for kw in [dict(n=4095), dict(cap=96), dict(q=120), dict(rb=8), dict(op_terms=40), dict(prec=_tp.TP_FP64)]:
        st, v = _query(**kw)
        assert st == _tp.TP_OK
        assert v > base, kw
    for kw in [dict(n=1023), dict(cap=20), dict(q=40)]:
        st, v = _query(**kw)
        assert st == _tp.TP_OK
        assert v < base, kw
    # a 2D problem of the same grid needs less than the 3D one
    assert _query(d=2)[1] < base
    # the sinc rule (more terms than the fit) needs more
    assert _query(method=_tp.TP_SYM_SINC, sinc_kl=60, sinc_kr=20)[1] > base


def test_workspace_query_covers_the_iteration_tensors():
    """A lower bound from the definition: the iteration holds eight Tucker tensors of the cap (core
    cap^d and d factors n x cap of the tensor precision), which the estimate must exceed."""
    for d, n, prec, cap in [(3, 2047, _tp.TP_MIXED, 50), (3, 2047, _tp.TP_FP64, 96), (2, 4095, _tp.TP_FP64, 64),
                            (3, 32767, _tp.TP_MIXED, 40)]:
        b = 8 if prec == _tp.TP_FP64 else 4
        tensors = 8 * (cap ** d + d * n * cap) * b
        st, v = _query(d=d, n=n, prec=prec, cap=cap)
        assert st == _tp.TP_OK
        assert v >= tensors, (d, n, prec, cap)


@pytest.mark.parametrize("kw", [dict(d=4), dict(d=1), dict(cap=0), dict(q=1), dict(rb=-1), dict(n=0)])
def test_workspace_query_rejects_out_of_range_sizes(kw):
    st, _ = _query(**kw)
    assert st == _tp.TP_EINVAL
    assert _err()


def test_batched_solve_argument_ranges():
    """tp_pcg_solve_batched checks count and streams before it touches the device."""
    lib = _lib()
    fake = C.c_void_p(1)  # never dereferenced: the range checks fail first
    desc = _tp._desc(3, 127, 0.5, 1.0, 1e-2, _tp.TP_MIXED, 28, 12)
    cp, t, sk = _tp.tp_cp(), _tp.tp_tensor(), _tp.tp_sketch()
    opts, info = _tp.tp_pcg_opts(), _tp.tp_pcg_info()
    args = (C.byref(desc), C.byref(cp), C.byref(t), C.byref(opts), C.byref(sk), C.byref(info))
    assert lib.tp_pcg_solve_batched(fake, -1, *args, 1, 0) == _tp.TP_EINVAL
    assert "count" in _err()
    for streams in (0, 17):
        assert lib.tp_pcg_solve_batched(fake, 1, *args, streams, 0) == _tp.TP_EINVAL
        assert "streams" in _err()


def test_missing_library_raises_instead_of_falling_back(monkeypatch, tmp_path):
    """With no built library the binding raises at load time: nothing in the package computes on
    the host in its place."""
    monkeypatch.setattr(_tp, "_LIB", None)
    monkeypatch.setattr(_tp, "library_path", lambda: str(tmp_path / "libtp.so"))
    with pytest.raises(OSError, match="not built"):
        _tp.load_library()


def test_package_sources_do_not_reach_the_oracle():
    """The product package (binding and HIP sources) names no module of the oracle: the oracle is
    test infrastructure only."""
    import re
    pkg = os.path.dirname(_tp.__file__)
    hits = []
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(root, f), errors="replace").read()
                if re.search(r"^\s*(from|import)\s+oracle\b|\boracle\.(exact|tensor|spectral|sinc|expfit|lowrank_pcg)\b",
                             src, flags=re.M):
                    hits.append(f)
    assert hits == []


def test_gemm_mode_range():
    """tp_gemm_mode takes 0, 1 or 2 (a process-wide switch, no device call) and rejects the rest."""
    lib = _lib()
    for bad in (-1, 3, 100):
        assert lib.tp_gemm_mode(bad) == _tp.TP_EINVAL
        assert "gemm mode" in _err()
    for ok in (2, 0, 1):
        assert lib.tp_gemm_mode(ok) == _tp.TP_OK
