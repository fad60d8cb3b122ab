"""Shared helpers of the GPU-vs-oracle parity tests (not a test module)."""
import os

import numpy as np

import oracle
import paper_1506_01418_amd as pkg

# Single-step tolerance for the FP32 path: |x_gpu - x_ref| <= TOL * c_x with
# c_x = |x_old| + eps (s_p G+_x + |prior'(x_old)|) + sigma R_x (the magnitude of
# every term that enters the update, computed by the oracle in FP64).
TOL_FP32 = 1e-5
# The dense blocks' BF16 path rounds the MFMA operands (W, H, E) to bfloat16.
TOL_BF16 = 2e-2


def bf16_round(x):
    """FP32 values rounded to the nearest bfloat16 (ties to even), returned
    as FP32: bfloat16 keeps the sign, the 8 exponent bits and the top 7
    mantissa bits of an FP32, so the candidates are the value with its low 16
    bits cleared and the next one up in magnitude."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    up = (low > 0x8000) | ((low == 0x8000) & (((u >> 16) & 1) == 1))
    r = ((u >> 16) + up.astype(np.uint64)) << 16
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(x))


def oracle_config(wl, flags=0, part_order="cyclic"):
    cfg = oracle.Config(**wl.fit_kwargs())
    cfg.flags = flags
    cfg.part_order = part_order
    return cfg


def scaled_error(x_gpu, x_ref, bound):
    d = np.abs(np.asarray(x_gpu, np.float64) - x_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(bound > 0, d / bound, np.where(d == 0, 0.0, np.inf))
    return e


def step_parity(wl, steps_before=0, flags=0, sampler=None, dense=False, **overrides):
    """Runs the GPU chain `steps_before` iterations, hands its FP32 state to
    the oracle, then takes one more iteration on both and returns the worst
    scaled error over W and H (and the sampler)."""
    kw = dict(dense_min_cols=1) if dense else {}   # keep narrow test blocks on the dense kernels
    kw.update(overrides)
    s = sampler or pkg.PSGLD.from_workload(wl, dense=dense, test_flags=flags, **kw)
    if steps_before:
        s.step(steps_before, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    Wg, Hg = s.factors()
    cfg = oracle_config(wl, flags, overrides.get("part_order", "cyclic"))
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol,
                      row_piece=overrides.get("row_piece"), col_piece=overrides.get("col_piece"))
    ch.set_state(Wg, Hg, s.iteration())
    bW, bH = ch.run(1, bounds=True)
    s.step(1, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    Wn, Hn = s.factors()
    eW = scaled_error(Wn, ch.W, bW)
    eH = scaled_error(Hn, ch.H, bH)
    return max(float(eW.max(initial=0)), float(eH.max(initial=0))), s


def philox_kat():
    """The published known-answer vectors of Philox4x32-10 (Salmon et al.,
    SC'11), from tests/golden: inputs (ctr0..3, key0..1) and outputs."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    rows = [[int(x, 16) for x in line.split()] for line in open(path) if line.strip() and line[0] != "#"]
    rows = np.array(rows, dtype=np.uint64).astype(np.uint32)
    assert rows.shape == (3, 10)
    return rows[:, :6], rows[:, 6:]
