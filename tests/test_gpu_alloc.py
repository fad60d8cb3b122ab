"""Device memory and streams supplied by the caller (options.dev_alloc /
dev_free / alloc_user and options.stream): a context whose every device
allocation comes from PyTorch's caching allocator and which runs on a
PyTorch stream computes bitwise what the library's own allocations and
stream compute; an allocator that returns NULL makes the call fail with
PSGLD_E_NOMEM and leaves nothing allocated."""
import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from test_gpu_dense import dense_case

pytestmark = pytest.mark.gpu


def _outputs(s):
    return (*s.factors(), *s.posterior_mean(), *s.posterior_var(), s.heldout_predictions(),
            np.array([s.num_samples(), s.iteration()]))


@pytest.mark.parametrize("dense", [False, True])
def test_torch_memory_and_stream_match_the_default_path(dense):
    import torch
    if dense:
        wl = dense_case(128, 600, 16, 2, 0.5, density=0.9, seed=91)
    else:
        wl = workloads.random_sparse(900, 500, 30_000, 16, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                     data_seed=93, chain_seed=94)
    wl.burn_in, wl.thin = 6, 2
    kw = dict(dense=dense, dense_min_cols=1) if dense else {}
    ref = pkg.PSGLD.from_workload(wl, **kw)
    stream = torch.cuda.Stream(device=0)            # default priority
    base = torch.cuda.memory_allocated(0)
    with torch.cuda.stream(stream):
        s = pkg.PSGLD.from_workload(wl, allocator="torch", **kw)
    assert s.stream() == stream.cuda_stream
    alloc = s.allocator
    assert alloc.bytes == s.memory_bytes() > 0
    assert torch.cuda.memory_allocated(0) - base >= alloc.bytes
    if not dense:
        for x in (ref, s):
            x.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(32,), iters=0)
    for n in (3, 17, 1):
        ref.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        s.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    for a, b in zip(_outputs(ref), _outputs(s)):
        assert np.array_equal(a, b, equal_nan=True)
    assert s.log_likelihood() == ref.log_likelihood()
    state = s.get_state()
    s.set_state(state)
    assert alloc.bytes == s.memory_bytes()
    s.close()
    ref.close()
    assert alloc.held == {}


@pytest.mark.parametrize("fail_after", [0, 3])
def test_allocator_returning_null_is_nomem(fail_after):
    wl = workloads.random_sparse(300, 220, 6000, 12, 4, data_seed=95, chain_seed=96)
    alloc = pkg.TorchAllocator(0, 0, fail_after=fail_after)
    s = pkg.PSGLD(wl.I, wl.J, wl.K, wl.B, allocator=alloc)
    with pytest.raises(pkg.PsgldError) as e:
        s.load_coo(wl.row, wl.col, wl.val)
    assert e.value.status == pkg.PSGLD_E_NOMEM, e.value
    assert "allocator hook returned NULL" in str(e.value)
    s.close()
    assert alloc.held == {}


def test_server_counts_bytes_through_the_hooks():
    """A server whose jobs allocate through PyTorch: while they run, the
    bytes the server charges them are bytes the hook handed out; results
    equal those of a server on the library's own allocations."""
    jobs = [workloads.serving_job(j, T=40, burn_in=20, max_side=600) for j in range(6)]
    out = []
    for allocator in (None, "torch"):
        srv = pkg.Server(1 << 30, max_active=8, iters_per_tick=10, allocator=allocator)
        ids = [srv.submit(wl, 40, dense=wl.dense is not None) for wl in jobs]
        charged = []
        while True:
            running, queued, _ = srv.tick()
            if allocator and running:
                charged.append((sum(srv.info(i)["bytes"] for i in ids), srv.allocator.bytes))
            if running == 0 and queued == 0:
                break
        out.append([srv.result(i) for i in ids])
        if allocator:
            assert charged and all(hook <= total for total, hook in charged)
            assert all(hook > 0 for _, hook in charged)
        srv.close()
        if allocator:
            assert srv.allocator.held == {}
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y), equal_nan=True)
