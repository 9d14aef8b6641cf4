"""The Python binding against the C header, without a GPU: the ctypes
structures must have the C compiler's layout (field order, offsets, sizes)
and the binding's constants the header's values,
and every function's ctypes argument list must match its prototype in
include/hmle.h in length and in the kind of each argument (pointer, 32-bit
integer or enum, 64-bit integer, float, double) and return type."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmle.h")


def _h():
    import paper_2104_07146_amd as h
    return h


def test_struct_layout_matches_c(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "abi_layout")
    b = subprocess.run([cc, "-std=c99", "-Wall", os.path.join(ROOT, "tests", "host", "abi_layout.c"), "-o", exe],
                       capture_output=True, text=True, timeout=120)
    assert b.returncode == 0, b.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout.split("\n")
    h = _h()
    py = {"hmle_theta": h.Theta, "hmle_opts": h.Opts, "hmle_fit_opts": h.FitOpts, "hmle_fit_report": h.FitReport,
          "hmle_tune_entry": h.TuneEntry}
    seen = {k: [] for k in py}
    for line in filter(None, out):
        s, f, off, size = line.split()
        if s == "const":
            assert getattr(h, f) == int(off), (f, getattr(h, f), off)
            continue
        cls = py[s]
        if f == "_size":
            assert ctypes.sizeof(cls) == int(off), (s, ctypes.sizeof(cls), off)
            continue
        seen[s].append(f)
        field = getattr(cls, f)
        assert (field.offset, field.size) == (int(off), int(size)), (s, f, field.offset, field.size, off, size)
    for s, cls in py.items():
        assert [f for f, _ in cls._fields_] == seen[s], s


_C_KIND = [
    (re.compile(r"\*|\[\s*\d*\s*\]"), "ptr"),
    (re.compile(r"\bint64_t\b"), "i64"),
    (re.compile(r"\b(int32_t|hmle_precision|hmle_status)\b"), "i32"),
    (re.compile(r"\bdouble\b"), "f64"),
    (re.compile(r"\bfloat\b"), "f32"),
    (re.compile(r"\b(hmle_problem|hmle_mlp)\b"), "ptr"),     # opaque handles are pointers
]


def _c_kind(decl: str) -> str:
    for pat, kind in _C_KIND:
        if pat.search(decl):
            return kind
    raise AssertionError(f"unknown C type in {decl!r}")


def _py_kind(t) -> str:
    if t is None:
        return "void"
    if t in (ctypes.c_void_p, ctypes.c_char_p) or issubclass(t, ctypes._Pointer):
        return "ptr"
    return {ctypes.c_int32: "i32", ctypes.c_int64: "i64", ctypes.c_double: "f64", ctypes.c_float: "f32"}[t]


def _prototypes():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"^\s*#.*$", " ", src, flags=re.M)        # preprocessor lines
    protos = {}
    for m in re.finditer(r"([A-Za-z_][\w\s\*]*?)\b(hmle_\w+)\s*\(([^;{]*?)\)\s*;", src):
        ret, name, args = m.group(1).strip(), m.group(2), m.group(3).strip()
        params = [] if args in ("", "void") else [a.strip() for a in args.split(",")]
        protos[name] = (ret, params)
    return protos


def test_argtypes_match_prototypes():
    h = _h()
    L = h.lib()
    protos = _prototypes()
    assert set(protos) == set(h.EXPORTED), set(protos) ^ set(h.EXPORTED)
    for name, (ret, params) in protos.items():
        fn = getattr(L, name)
        want = [_c_kind(p) for p in params]
        got = [_py_kind(t) for t in (fn.argtypes or [])]
        assert got == want, (name, got, want)
        if ret == "void":
            assert fn.restype is None, name
        elif ret == "int64_t":
            assert fn.restype is ctypes.c_int64, name
        elif "char" in ret:
            assert fn.restype is ctypes.c_char_p, name
        else:
            assert ret == "hmle_status" and fn.restype in (ctypes.c_int, ctypes.c_int32), (name, ret, fn.restype)
