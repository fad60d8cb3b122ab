"""Host-side checks of the C ABI that need no GPU: the library loads, every
function declared in include/psgld.h is exported, and argument validation of
psgld_create / psgld_load_coo happens on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1506_01418_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "psgld.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psgld_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 25
    L = C.CDLL(pkg.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pkg.SIGNATURES), set(names) ^ set(pkg.SIGNATURES)


def test_default_options():
    o = pkg.psgld_default_options()
    assert o.thin == 1 and o.dense_threshold == 0.3 and o.mu_floor == 1e-6 and o.device == 0
    assert o.graph_iters == -1 and o.persistent == 0 and o.part_order == pkg.PSGLD_PART_CYCLIC


@pytest.mark.parametrize("I,J,K,B,beta,phi,lw,msg", [
    (0, 5, 2, 1, 2.0, 1.0, 1.0, "I and J"),
    (5, 5, 0, 1, 2.0, 1.0, 1.0, "K must"),
    (5, 5, 300, 1, 2.0, 1.0, 1.0, "K must"),
    (5, 5, 2, 6, 2.0, 1.0, 1.0, "B must"),
    (5, 5, 2, 0, 2.0, 1.0, 1.0, "B must"),
    (5, 5, 2, 2, 2.0, 0.0, 1.0, "phi"),
    (5, 5, 2, 2, 1.5, 1.0, 1.0, "no Tweedie"),
    (5, 5, 2, 2, 2.0, 1.0, -1.0, "prior rates"),
])
def test_create_rejects_bad_arguments(I, J, K, B, beta, phi, lw, msg):
    with pytest.raises(pkg.PsgldError) as e:
        pkg.psgld_create(I, J, K, B, pkg.psgld_likelihood(beta, phi),
                         pkg.psgld_prior(pkg.PSGLD_PRIOR_GAUSSIAN, lw, 1.0, 0))
    assert e.value.status == pkg.PSGLD_E_ARG and msg in str(e.value)


def test_create_checks_pieces_and_thin():
    with pytest.raises(pkg.PsgldError, match="non-empty"):
        pkg.PSGLD(6, 6, 2, 3, row_piece=[0, 0, 1, 1, 1, 1])
    with pytest.raises(pkg.PsgldError, match="out of range"):
        pkg.PSGLD(6, 6, 2, 3, col_piece=[0, 0, 1, 1, 2, 3])
    with pytest.raises(pkg.PsgldError, match="thin"):
        pkg.PSGLD(6, 6, 2, 3, thin=0)


def test_load_validates_on_host_before_device():
    s = pkg.PSGLD(4, 4, 2, 2, beta=1.0, prior="exponential", mirror=True)
    with pytest.raises(pkg.PsgldError, match="out of range"):
        s.load_coo([0, 4], [0, 1], [1.0, 2.0])
    with pytest.raises(pkg.PsgldError, match="negative"):
        s.load_coo([0, 1], [0, 1], [1.0, -2.0])
    with pytest.raises(pkg.PsgldError, match="non-finite"):
        s.load_coo([0, 1], [0, 1], [1.0, np.nan])
    g = pkg.PSGLD(4, 4, 2, 2, beta=0.0)
    with pytest.raises(pkg.PsgldError, match="non-positive"):
        g.load_coo([0], [0], [0.0])
    # stepping before loading is a state error
    with pytest.raises(pkg.PsgldError) as e:
        s.step(1, 1e-3)
    assert e.value.status == pkg.PSGLD_E_STATE
    with pytest.raises(pkg.PsgldError) as e:
        pkg.psgld_step(s.ctx, 1, pkg.psgld_eps_schedule(1e-3, 1.0, 0.3))
    assert e.value.status == pkg.PSGLD_E_ARG
    # entry counts whose 32-bit entry indices (plus a batch and the padding
    # read past the last entry) would overflow are refused before any pointer
    # is read
    for nnz in (-1, 2**31 - 63, 2**31):
        with pytest.raises(pkg.PsgldError, match=r"nnz must be in \[0, 2\^31 - 64\]") as e:
            pkg._check(pkg.lib().psgld_load_coo(s.ctx, nnz, None, None, None), s.ctx)
        assert e.value.status == pkg.PSGLD_E_ARG
    s.close()
    g.close()


def test_balanced_pieces_lpt():
    """Heaviest first into the least-loaded piece: no piece empty, loads
    within the largest single weight of each other, deterministic."""
    rng = np.random.default_rng(5)
    w = (rng.zipf(1.3, 5000) % 20000).astype(np.int64)
    for B in (1, 3, 32, 64):
        p = pkg.psgld_balanced_pieces(w, B)
        loads = np.bincount(p, weights=w, minlength=B)
        assert np.all(np.bincount(p, minlength=B) > 0)
        assert loads.max() - loads.min() <= w.max()
        assert np.array_equal(p, pkg.psgld_balanced_pieces(w, B))
    # equal weights: sizes differ by at most one
    p = pkg.psgld_balanced_pieces(np.ones(103, np.int64), 10)
    sizes = np.bincount(p, minlength=10)
    assert sizes.max() - sizes.min() <= 1
    with pytest.raises(pkg.PsgldError):
        pkg.psgld_balanced_pieces(np.ones(3, np.int64), 4)
    with pytest.raises(pkg.PsgldError):
        pkg.psgld_balanced_pieces(np.array([1, -1, 2], np.int64), 2)


def test_balanced_pieces_even_out_zipf_parts():
    """On Zipf-skewed ratings the balanced pieces give parts of more equal
    size than contiguous pieces (smaller spread of s_p = N / n_p)."""
    import oracle
    wl = workloads_small_zipf()
    rp, cp = pkg.balanced_pieces_for(wl.row, wl.col, wl.I, wl.J, wl.B)
    def part_sizes(rp, cp):
        part = (cp[wl.col] - rp[wl.row]) % wl.B
        return np.bincount(part, minlength=wl.B)
    contiguous = part_sizes(oracle.partition(wl.I, wl.B), oracle.partition(wl.J, wl.B))
    balanced = part_sizes(rp, cp)
    assert balanced.max() / balanced.min() < contiguous.max() / contiguous.min()


def workloads_small_zipf():
    import workloads
    return workloads.random_sparse(3000, 800, 80_000, 8, 8, zipf_a=1.2, data_seed=17, chain_seed=18)


def test_default_options_have_no_allocator_hooks():
    o = pkg.psgld_default_options()
    assert o.persistent_grid == 0 and not o.dev_alloc and not o.dev_free and o.alloc_user is None


def test_create_rejects_one_allocator_hook_alone():
    alloc = pkg.DEV_ALLOC_FN(lambda n, u: None)
    free = pkg.DEV_FREE_FN(lambda p, n, u: None)
    lik = pkg.psgld_likelihood(2.0, 1.0)
    pr = pkg.psgld_prior(pkg.PSGLD_PRIOR_GAUSSIAN, 1.0, 1.0, 0)
    for a, f in [(alloc, None), (None, free)]:
        o = pkg.psgld_default_options()
        if a:
            o.dev_alloc = a
        if f:
            o.dev_free = f
        with pytest.raises(pkg.PsgldError, match="go together"):
            pkg.psgld_create(5, 5, 2, 1, lik, pr, o)
    o = pkg.psgld_default_options()
    o.persistent_grid = -1
    with pytest.raises(pkg.PsgldError, match="persistent_grid"):
        pkg.psgld_create(5, 5, 2, 1, lik, pr, o)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of psgld_options, psgld_server_options and psgld_job
    have the C header's field offsets and sizes (compiled with gcc here)."""
    structs = {"psgld_options": pkg.psgld_options, "psgld_server_options": pkg.psgld_server_options,
               "psgld_job": pkg.psgld_job}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "psgld.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_bf16_rounding_of_the_tests_is_nearest_even():
    """The tests' FP32 -> BF16 rounding (which stands in for the library's
    on the test side) against the definition: the nearest of all BF16 values,
    compared in exact FP64 arithmetic, ties to the even mantissa."""
    from parity import bf16_round
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * np.float32(1e3),
                        rng.gamma(0.5, 2.0, 20000).astype(np.float32),
                        np.float32([0.0, 1.0, 255.0, 256.0, 257.0, 3.0e38, 1e-30]),
                        # exact ties: 1 + 2^-8 (even below), 1 + 3 * 2^-8 (even above)
                        np.float32([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)])])
    r = bf16_round(x)
    u = x.view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo, dhi = np.abs(xd - lo), np.abs(hi - xd)
    lo_even = ((u >> np.uint32(16)) & np.uint32(1)) == 0
    want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo_even, lo, hi)))
    assert np.array_equal(r.astype(np.float64), want)
    assert np.all(r.view(np.uint32) & np.uint32(0xFFFF) == 0)
    assert r[-3] == np.float32(1.0) and r[-2] == np.float32(1.0 + 4 * 2.0 ** -8) and r[-1] == np.float32(-1.0)
    # integers up to 256 are BF16 values
    k = np.arange(257, dtype=np.float32)
    assert np.array_equal(bf16_round(k), k)


def test_c_program_builds_against_the_header(tmp_path):
    """A plain C user of the ABI (tests/c_abi_driver.c) compiles with
    -Wall -Werror against include/psgld.h and links to the in-tree library."""
    from c_driver import build_driver
    exe = build_driver(tmp_path)
    assert os.access(exe, os.X_OK)
