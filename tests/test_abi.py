"""The C ABI library loads and exports every symbol include/apr.h declares,
and the Python binding's structures match the C layout (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2409_11470_amd as A
    if not os.path.exists(A.lib_path()):
        import __graft_entry__
        __graft_entry__.build()
    return A.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_struct_layout_matches_header(tmp_path):
    import ctypes
    import paper_2409_11470_amd as A
    prog = tmp_path / "layout.c"
    fields = {"apr_params": [f for f, _ in A.Params._fields_],
              "apr_state": [f for f, _ in A.CState._fields_],
              "apr_zone": [f for f, _ in A.Zone._fields_],
              "apr_sink": [f for f, _ in A.Sink._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "apr.h"', 'int main(void){']
    for s, fs in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (s, s))
        for f in fs:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (s, f, s, f))
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for s, cls in (("apr_params", A.Params), ("apr_state", A.CState), ("apr_zone", A.Zone),
                   ("apr_sink", A.Sink)):
        assert int(out[s]) == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert int(out["%s.%s" % (s, f)]) == getattr(cls, f).offset, (s, f)


def test_constants_match_header(tmp_path):
    # every APR_ constant of the binding has the header's value (array sizes
    # such as APR_PROF_N size buffers the library writes into)
    import paper_2409_11470_amd._abi as B
    names = sorted(k for k in dir(B) if k.startswith("APR_") and isinstance(getattr(B, k), int))
    src = open(HEADER).read()
    assert all(n in src for n in names)
    prog = tmp_path / "consts.c"
    body = "".join('printf("%s %%ld\\n", (long)(%s));' % (n, n) for n in names)
    prog.write_text('#include <stdio.h>\n#include "apr.h"\nint main(void){%sreturn 0;}' % body)
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for n in names:
        assert int(out[n]) == getattr(B, n), n


def test_default_params(L):
    import paper_2409_11470_amd as A
    p = A.apr_default_params()
    assert p.hfact == 1.2 and p.r_sep_factor == 0.2 and p.nn_cap == 0.35
    assert p.precision == A.APR_FP32 and p.av_alpha == 1.0 and p.av_beta == 2.0


def test_invalid_params_rejected_without_gpu_work(L):
    import ctypes
    import paper_2409_11470_amd as A
    p = A.make_params(m0=-1.0)
    ptr = ctypes.c_void_p()
    assert L.apr_ctx_create(ctypes.byref(ptr), ctypes.byref(p), None) == A.APR_ERR_INVALID


def test_newton_iteration_limit_validated_without_gpu_work(L):
    # max_iter is 1 .. 1000 (the density kernel keeps each target's pass count
    # in 16 bits)
    import ctypes
    import paper_2409_11470_amd as A
    for bad in (0, 1001):
        p = A.make_params(m0=1.0, max_iter=bad)
        ptr = ctypes.c_void_p()
        assert L.apr_ctx_create(ctypes.byref(ptr), ctypes.byref(p), None) == A.APR_ERR_INVALID


def test_bench_refuses_several_gpus():
    # one GPU only: the multi-GPU request exits with a message before any GPU work
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
