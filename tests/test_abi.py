"""The C-ABI library loads without a GPU and exports every entry point that
include/qdwhp.h declares (no compute calls are made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdwhp.h")
LIB = os.path.join(ROOT, "paper_2104_14186_amd", "libqdwhp.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # drop comments
    return sorted(set(re.findall(r"\b(qdwhp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_solver_entry_points():
    names = declared()
    for must in ["qdwhp_eig", "qdwhp_svd", "qdwhp_eig_workspace", "qdwhp_svd_workspace",
                 "qdwhp_batched", "qdwhp_serve_create", "qdwhp_serve_submit", "qdwhp_serve_poll",
                 "qdwhp_serve_destroy", "qdwhp_dgemm_grouped", "qdwhp_tune_set"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, f"declared but not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    import paper_2104_14186_amd as q
    assert sorted(q.exported_symbols()) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    """Calls that touch no device: options, strings, tuning table, size queries."""
    import paper_2104_14186_amd as q
    L = q.lib()
    o = q.default_opts()
    assert o.tol == 0.05 and o.eig_iters == 3 and o.kappa_max == 100.0
    assert L.qdwhp_strerror(2)
    q.tune_set("test.key", 7)
    assert q.tune_get("test.key", -1) == 7
    assert q.tune_get("test.absent", 3) == 3
    assert L.qdwhp_eig_workspace(512, 0.1, ctypes.byref(o)) > 512 * 512 * 8
    # no graph captured yet: clearing touches no device
    assert L.qdwhp_graphs_count() == 0 and L.qdwhp_graphs_clear() == 0
    # k = floor(fraction n + 1/2) in [1, n]; 0 for arguments the solvers reject
    for n, f, k in ((16384, 0.2, 3277), (16384, 0.01, 164), (7, 0.5, 4), (10, 1e-9, 1), (10, 1.0, 10),
                    (10, 0.0, 0), (10, 1.5, 0), (0, 0.5, 0), (10, float("nan"), 0)):
        assert L.qdwhp_eig_count(n, f) == k, (n, f)
    # the binding reports a rejected fraction with the library's status
    with pytest.raises(q.QdwhpError) as e:
        q._count(10, 1.5)
    assert e.value.status == -4
    p = q.Problem()
    p.type, p.m, p.n, p.k = q.PROBLEM_SVD, 300, 200, 10
    assert L.qdwhp_problem_workspace(ctypes.byref(p), ctypes.byref(o)) == L.qdwhp_svd_workspace(300, 200, 10, ctypes.byref(o))
    probs = (q.Problem * 2)(p, p)
    assert L.qdwhp_batched_workspace(2, probs, ctypes.byref(o)) >= 2 * L.qdwhp_svd_workspace(300, 200, 10, ctypes.byref(o))
    # argument checks return before any device work
    assert L.qdwhp_eig(None, 4, 4, 0.5, 0, None, None, 4, None, 0, None, None, None) == -1
    assert L.qdwhp_batched(-1, None, None, 0, None, 0, None, None, None) == -1
    assert L.qdwhp_serve_submit(None, None, None) == -1


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of qdwhp_opts, qdwhp_info and qdwhp_problem have the
    size and field offsets that a C compiler gives the header's structs (a
    mismatch would let the library write past the caller's struct)."""
    import shutil
    import subprocess
    import paper_2104_14186_amd as q
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"qdwhp_opts": q.Opts, "qdwhp_info": q.Info, "qdwhp_problem": q.Problem}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qdwhp.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, what, val = line.split()
            got[(cname, what)] = int(val)
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def test_zolotarev_coefficients_match_the_oracle():
    """The library's host-side Zolotarev coefficients (Landen-chain elliptic
    functions in long double) against the oracle's (mpmath at 80 digits), down to
    l = 1e-16 where the modulus l' is within 1e-32 of 1."""
    import paper_2104_14186_amd as q
    from oracle.zolo import zolo_coeffs
    for l in [1e-16, 1e-12, 1e-8, 1e-4, 1e-2, 0.2, 0.5, 0.9, 0.999]:
        for r in [1, 2, 3, 5, 8, 13, 16]:
            a, b = q.zolo_coeffs(l, r), zolo_coeffs(l, r)
            assert np.max(np.abs(np.array(a["c"]) - b["c"]) / np.array(b["c"])) < 1e-15
            assert np.max(np.abs(np.array(a["a"]) - b["a"]) / np.abs(b["a"])) < 1e-15
            assert abs(a["M"] - b["M"]) < 1e-15 * b["M"]
            assert abs(a["l_next"] - b["l_next"]) < 1e-15
    with pytest.raises(RuntimeError):
        q.zolo_coeffs(1.0, 2)


def test_zolotarev_step_counts_match_the_oracle():
    """The step count depends on |Z(l) - 1| < 5u at the rounding level; the
    library's extended-precision l_next takes the oracle's decisions."""
    import paper_2104_14186_amd as q
    from oracle.zolo import zolo_schedule
    for s in [0.875, 0.2, 0.05, 1e-3, 1e-8, 1e-16]:
        for r in range(1, 17):
            l, k = s, 0
            while abs(l - 1.0) >= 5 * 2.0 ** -53 and k < 8:
                l = min(q.zolo_coeffs(min(l, 1 - 1e-16), r)["l_next"], 1.0)
                k += 1
            assert k == len(zolo_schedule(s, r)), (s, r)


def test_sized_tuning_lookup():
    """qdwhp_tune_get_sized: "key@b" with b = ceil(log2(size)) first, then "key",
    then the fallback (host-only calls)."""
    import paper_2104_14186_amd as q
    L = q.lib()
    old = {k: q.tune_get(k, -777) for k in ("zz.test", "zz.test@10")}
    try:
        q.tune_set("zz.test", 5)
        q.tune_set("zz.test@10", 9)
        assert L.qdwhp_tune_get_sized(b"zz.test", 1000, -1) == 9        # ceil(log2 1000) = 10
        assert L.qdwhp_tune_get_sized(b"zz.test", 1024, -1) == 9
        assert L.qdwhp_tune_get_sized(b"zz.test", 1025, -1) == 5        # bucket 11 unset
        assert L.qdwhp_tune_get_sized(b"zz.none", 1000, -3) == -3
    finally:
        L.qdwhp_tune_clear()
        q.load_tuning()
