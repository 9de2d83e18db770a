"""The C-ABI library loads and exports every entry point its header declares;
argument checks that need no device behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _lib_path():
    if os.environ.get("FRESCO_LIB"):
        return os.environ["FRESCO_LIB"]
    from paper_2305_15693_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    return B.LIB


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(fresco_[a-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["fresco_create", "fresco_destroy", "fresco_structure_factor",
                     "fresco_loss_grad", "fresco_error_string"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_without_device():
    lib = ctypes.CDLL(_lib_path())
    lib.fresco_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.fresco_create.restype = ctypes.c_int
    assert lib.fresco_create(None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.fresco_create(ctypes.byref(h), None, None) == -1
    assert h.value is None
    lib.fresco_destroy.argtypes = [ctypes.c_void_p]
    assert lib.fresco_destroy(None) == 0
    lib.fresco_error_string.restype = ctypes.c_char_p
    assert lib.fresco_error_string(-5) == b"non-finite position"
    for fn in ["fresco_structure_factor", "fresco_loss_grad", "fresco_loss_grad_async"]:
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
        assert f(None, None, None, None) == -1
    lib.fresco_set_timing_reps.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.fresco_set_timing_reps.restype = ctypes.c_int
    assert lib.fresco_set_timing_reps(None, 4) == -1
    lib.fresco_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.fresco_set_timing.restype = ctypes.c_int
    assert lib.fresco_set_timing(None, 1) == -1


def test_problem_validation_without_device():
    """Invalid problems are rejected before any device work."""
    from paper_2305_15693_amd import fresco as F
    lib = F.lib()

    def create(**kw):
        p = F.Problem()
        p.dim, p.dtype, p.n = 2, F.F32, 100
        p.box[0] = p.box[1] = 10.0
        p.kmax[0] = p.kmax[1] = 4
        p.k_cut, p.tol, p.upsampfac = 4.0, 1e-6, 2.0
        for k, v in kw.items():
            if k == "box":
                p.box[0] = v
            else:
                setattr(p, k, v)
        h = ctypes.c_void_p()
        return lib.fresco_create(ctypes.byref(h), ctypes.byref(p), None)

    assert create(dim=4) == F.EINVAL
    assert create(dtype=7) == F.EINVAL
    assert create(n=0) == F.EINVAL
    assert create(box=-1.0) == F.EINVAL
    assert create(tol=0.5) == F.EINVAL
    assert create(tol=0.0) == F.EINVAL
    assert create(upsampfac=1.25) == F.EINVAL
    assert create(weight_mode=9) == F.EINVAL
    assert create(n=1 << 40) == F.ENOTSUP


def test_binding_structs_match_the_header(tmp_path):
    # every struct the binding passes through the ABI has the header's size and
    # field offsets (compiled with the host C compiler; no device needed)
    import shutil
    import subprocess
    from paper_2305_15693_amd import fresco as F
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    structs = {"fresco_problem": F.Problem, "fresco_plan_info": F.PlanInfo,
               "fresco_pair_problem": F.PairProblem, "fresco_lbfgs_opts": F.LbfgsOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fresco.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    seen = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        seen[(cname, field)] = int(value)
    for cname, py in structs.items():
        assert seen[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert seen[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_algorithmic_bytes():
    # the per-launch bytes the roofline divides by, for the 2D headline workload
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_2305_15693_amd import inputs as I
    cfg = I.WORKLOADS["2d_n1e6_stealthy300_f32"]
    b = bench.stage_bytes(cfg, {"nf": [1250, 1250], "kmax": [300, 300]}, 4)
    N, nf, s = 10**6, 1250, 4
    assert b["spread"] == N * 2 * s + nf * nf * s
    assert b["interp"] == nf * nf * s + 2 * N * 2 * s
    assert b["fft_rows_fwd"] == nf * nf * s + nf * 301 * 8


def test_failed_creation_releases_everything():
    # without a device the first allocation fails: every create reports ENOMEM,
    # leaves *out NULL and releases what it had set up (run under the host
    # sanitizers too); with a device the objects are created and destroyed
    from paper_2305_15693_amd import fresco as F
    lib = F.lib()
    p = F.Problem()
    p.dim, p.dtype, p.n = 2, F.F32, 100
    p.box[0] = p.box[1] = 10.0
    p.kmax[0] = p.kmax[1] = 4
    p.k_cut, p.tol, p.upsampfac = 4.0, 1e-6, 2.0
    pp = F.PairProblem()
    pp.dim, pp.dtype, pp.n = 2, F.F32, 100
    pp.box[0] = pp.box[1] = 10.0
    pp.sigma, pp.eps, pp.alpha = 0.5, 1.0, 2.0
    batch = (F.Problem * 2)(p, p)
    calls = [(lib.fresco_create, (ctypes.byref(p),), lib.fresco_destroy),
             (lib.fresco_pair_create, (ctypes.byref(pp),), lib.fresco_pair_destroy),
             (lib.fresco_batch_create, (2, batch), lib.fresco_batch_destroy)]
    for create, args, destroy in calls:
        h = ctypes.c_void_p()
        st = create(ctypes.byref(h), *args, None)
        if st == F.OK:
            assert h.value is not None
            assert destroy(h) == F.OK
        else:
            assert st == F.ENOMEM
            assert h.value is None


def _generated_eval_ops(width, fn):
    """(FMAs, products) of one kernel-value function in the generated FP32 header."""
    from paper_2305_15693_amd import build as B
    path = os.path.join(B.OBJDIR, "kernel_tables.h")
    if not os.path.exists(path):
        B._generate_tables()
    text = open(path).read()
    body = text[text.index("struct Poly<%d> {" % width):]
    body = body[body.index(" void %s(float x" % fn):]
    body = body[:body.index("\n  }\n")]
    return body.count("fmaf("), body.count(" * ")


def test_bench_algorithmic_flops():
    # the per-point flops the ALU roofline divides by: the kernel values as the
    # generated evaluators compute them (operations counted in the generated
    # header) and the tensor-product contraction
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_2305_15693_amd import inputs as I
    ops = {}
    for w, fn in ((7, "es"), (8, "ch"), (8, "dch")):
        fm, mul = _generated_eval_ops(w, fn)
        ops[fn] = 2 * fm + mul
        assert bench.kernel_eval_flops(w) == ops[fn], (w, fn, fm, mul)
    cfg = I.WORKLOADS["2d_n1e6_stealthy300_f32"]
    f = bench.stage_flops(cfg, {"width": 7})
    wi = 8
    # the derivative shares y = x^2 with the kernel value
    both = ops["ch"] + ops["dch"] - 1
    assert f["per_point"]["interp"] == 2 * both + 2 * (2 * wi * wi + 3 * wi) == 626
    assert f["per_point"]["spread"] == 2 * ops["es"] + 7 + 49
    cfg3 = I.WORKLOADS["3d_n1e7_stealthy60_f32"]
    f3 = bench.stage_flops(cfg3, {"width": 7})
    assert f3["per_point"]["interp"] == 3 * both + 2 * (2 * wi ** 3 + 3 * wi ** 2 + 4 * wi)
    assert f3["interp"] == 10_000_000 * f3["per_point"]["interp"]
    assert abs(bench.ALU_PEAK_TFLOPS - 78.6432) < 1e-3
