"""CPU checks of the C ABI: the library loads, exports every function that
include/cprand.h declares, and rejects invalid arguments before any HIP
call (so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cprand.h")

P = pytest.importorskip("paper_1701_06600_amd")
from paper_1701_06600_amd import _abi  # noqa: E402


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(cprand_[a-z0-9_]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared_functions()
    assert "cprand_mttkrp_sampled" in names and "cprand_als" in names
    bound = {n for n, _, _ in _abi.SIGNATURES}
    for n in names:
        assert hasattr(P._lib, n), n
        assert n in bound, "no ctypes signature for %s" % n


def test_version_and_strerror():
    assert P.cprand_version().startswith("cprand-gfx950")
    for code in (0, 1, 2, 4, -1, -2, -3, -4, -5):
        assert P._lib.cprand_strerror(code)


def _tensor(order=3, dims=(4, 5, 6), dtype=_abi.F32, data=1):
    t = _abi.cprand_tensor()
    t.order = order
    t.dtype = dtype
    s = 1
    for i in range(order):
        t.dims[i] = dims[i] if i < len(dims) else 1
        t.strides[i] = s
        s *= t.dims[i]
    t.data = data
    return t


def test_sample_validation():
    L = P._lib
    dims = (C.c_int64 * 3)(4, 5, 6)
    assert L.cprand_sample(1, dims, 0, 10, 0, 0, None, None, None, None) == P.EINVAL
    assert L.cprand_sample(9, dims, 0, 10, 0, 0, None, None, None, None) == P.EINVAL
    assert L.cprand_sample(3, dims, 3, 10, 0, 0, None, C.c_void_p(16), None, None) == P.EINVAL
    assert L.cprand_sample(3, dims, 0, 0, 0, 0, None, C.c_void_p(16), None, None) == P.EINVAL
    assert L.cprand_sample(3, dims, 0, 10, 0, 0, None, None, None, None) == P.EINVAL
    bad = (C.c_int64 * 3)(4, 0, 6)
    assert L.cprand_sample(3, bad, 0, 10, 0, 0, None, C.c_void_p(16), None, None) == P.EINVAL
    assert b"dims" in L.cprand_last_error()


def test_mttkrp_validation():
    L = P._lib
    X = _tensor()
    A = (C.c_void_p * 3)(16, 16, 16)
    ws = C.c_void_p(16)
    # rank outside [1, 64]
    assert L.cprand_mttkrp_sampled(C.byref(X), 0, A, 65, 10, C.c_void_p(16), None, None, C.c_void_p(16),
                                   C.c_void_p(16), ws, 1 << 30, None) == P.EINVAL
    # mode out of range
    assert L.cprand_mttkrp_sampled(C.byref(X), 3, A, 4, 10, C.c_void_p(16), None, None, C.c_void_p(16),
                                   C.c_void_p(16), ws, 1 << 30, None) == P.EINVAL
    # workspace too small
    assert L.cprand_mttkrp_sampled(C.byref(X), 0, A, 4, 10, C.c_void_p(16), None, None, C.c_void_p(16),
                                   C.c_void_p(16), ws, 8, None) == P.EINVAL
    # mixed tensor without unmix signs
    Xc = _tensor(dtype=_abi.C64)
    assert L.cprand_mttkrp_sampled(C.byref(Xc), 0, A, 4, 10, C.c_void_p(16), None, None, C.c_void_p(16),
                                   C.c_void_p(16), ws, 1 << 30, None) == P.EINVAL
    # bad dtype and order
    assert L.cprand_mttkrp_sampled(C.byref(_tensor(dtype=9)), 0, A, 4, 10, C.c_void_p(16), None, None,
                                   C.c_void_p(16), C.c_void_p(16), ws, 1 << 30, None) == P.EINVAL
    assert L.cprand_mttkrp_sampled(C.byref(_tensor(order=1)), 0, A, 4, 10, C.c_void_p(16), None, None,
                                   C.c_void_p(16), C.c_void_p(16), ws, 1 << 30, None) == P.EINVAL


def test_mttkrp_noalloc_validation():
    """The fixed-scratch entry point rejects, before any HIP call, what the
    workspace one rejects, mixed tensors, and shapes whose partials exceed
    its array."""
    L = P._lib
    A = (C.c_void_p * 3)(16, 16, 16)
    args = (C.c_void_p(16), None, C.c_void_p(16), C.c_void_p(16), None)
    assert L.cprand_mttkrp_sampled_noalloc(C.byref(_tensor()), 0, A, 65, 10, *args) == P.EINVAL
    assert L.cprand_mttkrp_sampled_noalloc(C.byref(_tensor()), 3, A, 4, 10, *args) == P.EINVAL
    assert L.cprand_mttkrp_sampled_noalloc(C.byref(_tensor(dtype=_abi.C64)), 0, A, 4, 10, *args) == P.EUNSUPPORTED
    big = _tensor(dims=(1 << 24, 8, 8))
    assert L.cprand_mttkrp_sampled_noalloc(C.byref(big), 0, A, 64, 4096, *args) == P.EINVAL
    assert b"scratch" in L.cprand_last_error()


def test_workspace_size_monotone_and_zero_on_bad_args():
    X = _tensor(dims=(400, 400, 400))
    a = P._lib.cprand_workspace_size(C.byref(X), 10, 300, 2 ** 14)
    b = P._lib.cprand_workspace_size(C.byref(X), 10, 3000, 2 ** 14)
    assert 0 < a <= b
    assert P._lib.cprand_workspace_size(C.byref(X), 0, 300, 10) == 0
    assert P._lib.cprand_workspace_size(C.byref(X), 10, 0, 10) == 0


def test_solve_fit_mix_layout_validation():
    L = P._lib
    p16 = C.c_void_p(16)
    assert L.cprand_solve(0, 4, p16, p16, _abi.F64, None, None, p16, p16, None, p16, 1 << 20, None) == P.EINVAL
    assert L.cprand_solve(10, 4, p16, p16, _abi.BF16, None, None, p16, p16, None, p16, 1 << 20, None) == P.EINVAL
    assert L.cprand_solve(10, 4, p16, p16, _abi.F64, None, None, p16, p16, None, p16, 8, None) == P.EINVAL
    X = _tensor()
    A = (C.c_void_p * 3)(16, 16, 16)
    assert L.cprand_fit_est(C.byref(X), p16, A, p16, 4, 0, 1, p16, p16, 1 << 20, None) == P.EINVAL
    Xh = _tensor(dtype=_abi.C128)
    assert L.cprand_mix(C.byref(X), 1, C.byref(Xh), p16, p16, p16, 1 << 20, None) == P.EINVAL
    assert L.cprand_mix_factor(50, 5, p16, _abi.BF16, p16, p16, 0, None) == P.EINVAL
    out = (C.c_int64 * 3)()
    assert L.cprand_mode_major_strides(3, (C.c_int64 * 3)(5, 6, 7), 1, 8, out) == 0
    assert tuple(out) == (8, 1, 40)
    assert L.cprand_mode_major_strides(3, (C.c_int64 * 3)(5, 6, 7), 1, 4, out) == P.EINVAL


def test_plan_validation():
    X = _tensor()
    o = P.make_opts(R=0, S=10)
    h = C.c_void_p()
    assert P._lib.cprand_plan_create(C.byref(X), C.byref(o), C.byref(h)) == P.EINVAL
    o = P.make_opts(R=4, S=10, precision=P.PREC_BF16_REFINE)
    Xd = _tensor(dtype=_abi.F64)
    assert P._lib.cprand_plan_create(C.byref(Xd), C.byref(o), C.byref(h)) == P.EINVAL
    o = P.make_opts(R=4, S=10, proposal=P.PROPOSAL_TABLE)
    assert P._lib.cprand_plan_create(C.byref(X), C.byref(o), C.byref(h)) == P.EINVAL


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    that a C compiler gives the structures of include/cprand.h."""
    structs = [_abi.cprand_tensor, _abi.cprand_opts, _abi.cprand_report]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "cprand.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append('    printf("%s sizeof %%zu\\n", sizeof(%s));' % (n, n))
        for f in st._fields_:
            lines.append('    printf("%s %s %%zu\\n", offsetof(%s, %s));' % (n, f[0], n, f[0]))
    lines.append("    return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(l.split()[0], l.split()[1]): int(l.split()[2]) for l in out if l.strip()}
    for st in structs:
        n = st.__name__
        assert got[(n, "sizeof")] == C.sizeof(st), n
        for f in st._fields_:
            assert got[(n, f[0])] == getattr(st, f[0]).offset, (n, f[0])


def _header_defines():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, val in re.findall(r"#define\s+CPRAND_([A-Z0-9_]+)\s+\(?(-?\d+)\)?", text):
        out[name] = int(val)
    return out


def test_binding_constants_match_header_defines():
    """Every constant the binding passes across the ABI is #defined in the
    header with the same value."""
    d = _header_defines()
    names = ["MAX_ORDER", "MAX_RANK", "OK", "W_PINV", "W_MAXIT", "W_FALLBACK", "EINVAL", "ENAN", "EHIP",
             "ENOMEM", "EUNSUPPORTED", "F64", "F32", "BF16", "C64", "C128", "MIX_NONE", "MIX_FFT", "MIX_DCT",
             "PREC_NATIVE", "PREC_BF16_REFINE", "PREC_BF16", "PROPOSAL_UNIFORM", "PROPOSAL_TABLE",
             "PROPOSAL_LEARNED", "PROPOSAL_MARGINAL", "PROPOSAL_MIXTURE", "PROPOSAL_LEVERAGE",
             "NOALLOC_SCRATCH_BYTES"]
    for n in names:
        assert n in d, "CPRAND_%s is not #defined in the header" % n
        assert getattr(_abi, n) == d[n], (n, getattr(_abi, n), d[n])
    # and nothing the header defines is missing from the binding
    for n in d:
        assert hasattr(_abi, n), "CPRAND_%s has no binding constant" % n
