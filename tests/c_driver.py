"""Builds and feeds tests/c_abi_driver.c, a plain C user of the library's
ABI (test infrastructure, not a test module)."""
import os
import subprocess

import numpy as np

import paper_1506_01418_amd as pkg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def build_driver(out_dir):
    """gcc -> <out_dir>/c_abi_driver, linked to the in-tree libpsgld.so."""
    exe = os.path.join(str(out_dir), "c_abi_driver")
    lib_dir = os.path.dirname(pkg.LIB_PATH)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "c_abi_driver.c"), "-o", exe, "-L", lib_dir, "-l:libpsgld.so",
           f"-Wl,-rpath,{lib_dir}", "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def write_problem(d, wl):
    prior = 0 if wl.prior == "exponential" else 1
    with open(os.path.join(str(d), "problem.txt"), "w") as f:
        f.write(f"{wl.I} {wl.J} {wl.K} {wl.B} {wl.beta!r} {wl.phi!r} {prior} {wl.lambda_w!r} {wl.lambda_h!r} "
                f"{int(bool(wl.mirror))} {wl.seed} {wl.eps_a!r} {wl.eps_t0!r} {wl.eps_gamma!r} {len(wl.row)}\n")
    for name, a, dt in (("row.i32", wl.row, np.int32), ("col.i32", wl.col, np.int32), ("val.f32", wl.val, np.float32),
                        ("W0.f32", wl.W0, np.float32), ("H0.f32", wl.H0, np.float32)):
        np.ascontiguousarray(a, dtype=dt).tofile(os.path.join(str(d), name))


def run_driver(exe, d, n_iter, wl, timeout=120):
    """Runs the driver; returns (W, H, mean W, mean H) read back (means None
    for n_iter = 0)."""
    subprocess.run([exe, str(d), str(n_iter)], check=True, capture_output=True, text=True, timeout=timeout)
    W = np.fromfile(os.path.join(str(d), "W.f32"), dtype=np.float32).reshape(wl.I, wl.K)
    H = np.fromfile(os.path.join(str(d), "H.f32"), dtype=np.float32).reshape(wl.K, wl.J)
    if n_iter == 0:
        return W, H, None, None
    mW = np.fromfile(os.path.join(str(d), "mean_W.f64"), dtype=np.float64).reshape(wl.I, wl.K)
    mH = np.fromfile(os.path.join(str(d), "mean_H.f64"), dtype=np.float64).reshape(wl.K, wl.J)
    return W, H, mW, mH
