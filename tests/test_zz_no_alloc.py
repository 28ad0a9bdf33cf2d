"""smc_delta_e64_noalloc (the FP64 probe without any allocation, for callers that cannot
allocate) against smc_delta_e64 and the oracle, through the C ABI.

Two calls in a row on one stream share the library's fixed work space; the second is smaller
than the first (which fills the work space to its limit), so it must not see the first call's
entries.  Both must equal smc_delta_e64 bit for bit (the same proposals and FP64 evaluator) and
the oracle's dE within 1e-9 eV on sampled trials."""
import numpy as np
import pytest

import oracle
from gpu_common import make, need_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_probe_equals_probe_on_two_calls():
    torch = need_gpu()
    import paper_2604_08250_amd as smc
    from paper_2604_08250_amd import _lib as L
    print("[gpu-test] no-alloc probe: 16x16x16 cells, calls of 8192 then 3000 trials", flush=True)
    cells = (16, 16, 16)
    w, mc, model, occ = make("c2", cells=cells)
    mc.sweep(2)
    state = mc.occ.cpu().numpy()
    sweep = mc.sweep_index
    cap = 8192  # SMC_NOALLOC_MAX_TRIALS in include/smc.h
    rng = np.random.default_rng(8)
    calls = [rng.permutation(mc.n_sites)[:cap], rng.choice(mc.n_sites, size=3000, replace=False)]
    outs = []
    for sites in calls:
        s_dev = torch.as_tensor(sites, dtype=torch.int64, device="cuda")
        p_dev = torch.full((sites.size,), -7, dtype=torch.int64, device="cuda")
        e_dev = torch.full((sites.size,), float("nan"), dtype=torch.float64, device="cuda")
        L.smc_delta_e64_noalloc(mc.ctx, 0, sweep, s_dev.data_ptr(), sites.size, p_dev.data_ptr(), e_dev.data_ptr())
        outs.append((s_dev, p_dev, e_dev))
    torch.cuda.synchronize()
    for sites, (_, p_dev, e_dev) in zip(calls, outs):
        p_ref, e_ref = mc.delta_e64(sites, sweep=sweep)
        p, e = p_dev.cpu().numpy(), e_dev.cpu().numpy()
        assert np.array_equal(p, p_ref)
        assert np.array_equal(e, e_ref)  # bit for bit: same entries, same evaluator
        for k in rng.choice(sites.size, size=6, replace=False):
            rec = oracle.trial(cells, model, state, w.temperatures[0], w.seed, 0, sweep, int(sites[k]))
            assert rec["partner"] == p[k]
            assert abs(rec["dE"] - e[k]) < 1e-9
    # the probe changes nothing
    assert np.array_equal(mc.occ.cpu().numpy(), state)
    mc.close()


def test_noalloc_probe_limits():
    torch = need_gpu()
    from paper_2604_08250_amd import _lib as L
    print("[gpu-test] no-alloc probe: limits and sites outside the replica", flush=True)
    w, mc, model, occ = make("c2", cells=(8, 8, 8))
    dummy = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(L.SMCError):
        L.smc_delta_e64_noalloc(mc.ctx, 0, 0, dummy.data_ptr(), 8193, 0, dummy.data_ptr())
    with pytest.raises(L.SMCError):
        L.smc_delta_e64_noalloc(mc.ctx, 1, 0, dummy.data_ptr(), 1, 0, dummy.data_ptr())
    L.smc_delta_e64_noalloc(mc.ctx, 0, 0, 0, 0, 0, 0)  # n = 0: nothing to do
    # sites outside the replica are caught by the kernel's bounds check: partner -1, dE NaN
    sites = np.array([5, -1, mc.n_sites, 17], dtype=np.int64)
    s_dev = torch.as_tensor(sites, device="cuda")
    p_dev = torch.zeros(4, dtype=torch.int64, device="cuda")
    e_dev = torch.zeros(4, dtype=torch.float64, device="cuda")
    L.smc_delta_e64_noalloc(mc.ctx, 0, 0, s_dev.data_ptr(), 4, p_dev.data_ptr(), e_dev.data_ptr())
    torch.cuda.synchronize()
    p, e = p_dev.cpu().numpy(), e_dev.cpu().numpy()
    p_ref, e_ref = mc.delta_e64(sites[[0, 3]], sweep=0)
    assert p[1] == -1 and p[2] == -1 and np.isnan(e[1]) and np.isnan(e[2])
    assert np.array_equal(p[[0, 3]], p_ref) and np.array_equal(e[[0, 3]], e_ref)
    mc.close()
