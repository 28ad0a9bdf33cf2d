"""Differentiation pattern on the GPU, through the C ABI: cluster-expansion labels, snapshot
energies and their hand-written backward, the autograd wrapper, and the fused fit step.

Bar (FP64 reference mode): energies within 1e-9 relative of the oracle, gradients equal to the
oracle's FP64 gradient up to the FP32 rounding of the output, and to central differences of
the GPU's own FP64 forward.  FP32 mode: relative gradient error below 1e-5.  BF16 matrix-core
mode: gradient within 1e-4 (relative norm) of a CPU emulation of the same quantised arithmetic
and within 5e-2 of the FP64 gradient.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _ctx(precision, params):
    """A fit context: the lattice it carries is irrelevant to the fit calls (4^3 cells)."""
    import paper_2604_08250_amd as smc
    occ = synth.random_occupancy(4, 4, None, seed=0)
    return smc.SwapMC([(4, 4, 4)], [1000.0], occ, params, n_species=4, feature=1, hidden=128,
                      precision=precision, seed=0)


def _ce():
    p = synth.ce_params()
    tri = oracle.ce_triangles()
    return p, oracle.CEModel(p["n_species"], p["pair"], tri[p["triangle"]], p["species"], p["J"])


def _params(seed=11):
    return synth.mlp_params(108, 128, seed=seed)


def test_ce_energy_matches_oracle():
    torch = need_gpu()
    from paper_2604_08250_amd.fit import ce_energy
    p, ce = _ce()
    mc = _ctx("fp32", _params())
    for L in (4, 5, 8):
        _banner(f"CE labels L={L}")
        snaps = synth.snapshots(3, L, seed=30 + L)
        got = ce_energy(mc, p, torch.from_numpy(snaps).cuda(), L).cpu().numpy()
        want = np.array([oracle.ce_total((L, L, L), ce, s) for s in snaps])
        assert np.allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())
    mc.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reference_fwd_bwd_match_oracle(precision):
    torch = need_gpu()
    from paper_2604_08250_amd._lib import smc_energy_bwd, smc_energy_fwd
    params = _params()
    model = oracle.MLP(1, 128, params)
    mc = _ctx(precision, params)
    L = 4
    snaps = synth.snapshots(3, L, seed=40)
    gE = np.array([0.7, -1.3, 0.25])
    _banner(f"reference fwd/bwd {precision}")
    S_or = oracle.snapshot_energies((L, L, L), model, snaps)
    g_or = oracle.energy_grad((L, L, L), model, snaps, gE)
    d_snaps = torch.from_numpy(snaps).cuda()
    d_p = torch.from_numpy(params).cuda()
    S = torch.empty(3, dtype=torch.float64, device="cuda")
    smc_energy_fwd(mc.ctx, d_snaps.data_ptr(), 3, L, d_p.data_ptr(), S.data_ptr())
    d_g = torch.from_numpy(gE).cuda()
    grad = torch.empty_like(d_p)
    smc_energy_bwd(mc.ctx, d_snaps.data_ptr(), 3, L, d_p.data_ptr(), d_g.data_ptr(), grad.data_ptr())
    S, grad = S.cpu().numpy(), grad.cpu().numpy().astype(np.float64)
    if precision == "fp64":
        assert np.allclose(S, S_or, rtol=1e-12, atol=0)
        # FP64 throughout, then rounded to FP32 on output
        assert np.all(np.abs(grad - g_or) <= 2 ** -23 * np.abs(g_or) + 1e-30)
    else:
        assert np.allclose(S, S_or, rtol=2e-6, atol=0)
        rel = np.linalg.norm(grad - g_or) / np.linalg.norm(g_or)
        _banner(f"fp32 gradient relative error {rel:.2e}")
        assert rel < 1e-5
    # deterministic: a second call gives identical bits
    grad2 = torch.empty_like(d_p)
    smc_energy_bwd(mc.ctx, d_snaps.data_ptr(), 3, L, d_p.data_ptr(), d_g.data_ptr(), grad2.data_ptr())
    assert np.array_equal(grad2.cpu().numpy().astype(np.float64), grad)
    mc.close()


def test_fp64_gradient_matches_central_differences_of_gpu_forward():
    """1,000 parameters (FD seed): (S(p + h) - S(p - h)) / (stored difference), FP64 forward."""
    torch = need_gpu()
    from paper_2604_08250_amd._lib import smc_energy_bwd, smc_energy_fwd
    params = _params()
    mc = _ctx("fp64", params)
    L, B = 4, 2
    snaps = torch.from_numpy(synth.snapshots(B, L, seed=41)).cuda()
    gE = torch.tensor([1.0, -0.5], dtype=torch.float64, device="cuda")
    p = torch.from_numpy(params).cuda()
    grad = torch.empty_like(p)
    smc_energy_bwd(mc.ctx, snaps.data_ptr(), B, L, p.data_ptr(), gE.data_ptr(), grad.data_ptr())
    grad = grad.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(synth.SEED_FD)
    idx = rng.choice(params.size, size=1000, replace=False)
    S = torch.empty(B, dtype=torch.float64, device="cuda")
    _banner("FD on 1000 parameters")
    worst = 0.0
    for k in idx:
        vals = []
        stored = []
        for sgn in (1.0, -1.0):
            q = p.clone()
            v = np.float32(params[k] + sgn * 1e-4 * max(1.0, abs(float(params[k]))))
            q[int(k)] = float(v)
            stored.append(float(v))
            smc_energy_fwd(mc.ctx, snaps.data_ptr(), B, L, q.data_ptr(), S.data_ptr())
            vals.append(float((S * gE).sum()))
        fd = (vals[0] - vals[1]) / (stored[0] - stored[1])
        err = abs(fd - grad[k])
        worst = max(worst, err / (abs(grad[k]) + 1e-3))
        # central difference error ~ h^2 f'''/6 with h = 1e-4, FP64 rounding of S over 2h, and
        # the FP32 rounding (2^-24) of the returned gradient
        assert err <= 1e-5 * abs(grad[k]) + 1e-6, (k, fd, grad[k])
    _banner(f"worst scaled FD error {worst:.2e}")
    mc.close()


@pytest.mark.parametrize("L,B", [(4, 4), (5, 3), (6, 2)])
def test_bf16_fwd_bwd_match_emulation_and_fp64(L, B):
    """BF16 energies and gradient against the CPU emulation of the same quantisation points
    and against FP64.  4^3 cells: one 128-row chunk per snapshot; 5^3: a chunk that runs past
    the snapshot's last site; 6^3 with two snapshots: each snapshot split into segments over
    several blocks, the last chunk partial."""
    torch = need_gpu()
    import emulate
    from paper_2604_08250_amd._lib import smc_energy_bwd, smc_energy_fwd
    params = _params()
    model = oracle.MLP(1, 128, params)
    cells = (L, L, L)
    snaps = synth.snapshots(B, L, seed=42)
    gE = np.array([0.9, -0.4, 1.7, -1.1])[:B]
    mc = _ctx("bf16", params)
    d_snaps = torch.from_numpy(snaps).cuda()
    d_p = torch.from_numpy(params).cuda()
    S = torch.empty(B, dtype=torch.float64, device="cuda")
    smc_energy_fwd(mc.ctx, d_snaps.data_ptr(), B, L, d_p.data_ptr(), S.data_ptr())
    grad = torch.empty_like(d_p)
    d_g = torch.from_numpy(gE).cuda()
    smc_energy_bwd(mc.ctx, d_snaps.data_ptr(), B, L, d_p.data_ptr(), d_g.data_ptr(), grad.data_ptr())
    S, grad = S.cpu().numpy(), grad.cpu().numpy().astype(np.float64)
    X = emulate.snapshot_rows(cells, snaps)
    N = snaps.shape[1]
    S_emu = emulate.energies(params, X, "bf16").reshape(B, N).sum(axis=1)
    S_64 = oracle.snapshot_energies(cells, model, snaps)
    _banner(f"bf16 L={L} B={B}: S - emu {np.abs(S - S_emu).max():.3e}, S - fp64 {np.abs(S - S_64).max():.3e}")
    assert np.allclose(S, S_emu, rtol=0, atol=1e-4 * N)
    g_emu = emulate.fit_grad_bf16(params, X, np.repeat(gE, N))
    g_64 = oracle.energy_grad(cells, model, snaps, gE)
    r_emu = np.linalg.norm(grad - g_emu) / np.linalg.norm(g_emu)
    r_64 = np.linalg.norm(grad - g_64) / np.linalg.norm(g_64)
    _banner(f"bf16 L={L} B={B} gradient: rel err vs emulation {r_emu:.2e}, vs fp64 {r_64:.2e}")
    # same quantisation points: differences come from FP32 accumulation order and the rare
    # BF16 rounding flip it causes
    assert r_emu < 1e-4
    assert r_64 < 5e-2
    # block-wise: each parameter group agrees with the emulation on its own scale
    H, F = 128, 108
    bounds = [0, H * F, H * F + H, H * F + H + H * H, H * F + 2 * H + H * H, H * F + 3 * H + H * H, params.size]
    for a, b in zip(bounds[:-1], bounds[1:]):
        e = np.linalg.norm(grad[a:b] - g_emu[a:b]) / (np.linalg.norm(g_emu[a:b]) + 1e-30)
        assert e < 1e-3, (a, b, e)
    grad2 = torch.empty_like(d_p)
    smc_energy_bwd(mc.ctx, d_snaps.data_ptr(), B, L, d_p.data_ptr(), d_g.data_ptr(), grad2.data_ptr())
    assert np.array_equal(grad2.cpu().numpy().astype(np.float64), grad)
    mc.close()


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_autograd_function(precision):
    """torch autograd through SnapshotEnergy: the loss gradient equals the oracle's."""
    torch = need_gpu()
    from paper_2604_08250_amd.fit import snapshot_energy
    params = _params()
    model = oracle.MLP(1, 128, params)
    L, B = 4, 3
    cells = (L, L, L)
    snaps = synth.snapshots(B, L, seed=43)
    _, ce = _ce()
    labels = np.array([oracle.ce_total(cells, ce, s) for s in snaps])
    mc = _ctx(precision, params)
    p = torch.from_numpy(params).cuda().requires_grad_(True)
    S = snapshot_energy(mc, p, torch.from_numpy(snaps).cuda(), L)
    N = snaps.shape[1]
    loss = (((S - torch.from_numpy(labels).cuda()) / N) ** 2).mean()
    loss.backward()
    l_or, _, g_or = oracle.fit_loss_grad(cells, model, snaps, labels)
    g = p.grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - g_or) / np.linalg.norm(g_or)
    _banner(f"autograd {precision}: loss {float(loss):.6e} vs {l_or:.6e}, grad rel err {rel:.2e}")
    if precision == "fp64":
        assert float(loss) == pytest.approx(l_or, rel=1e-10)
        assert rel < 1e-6
    else:
        assert float(loss) == pytest.approx(l_or, rel=0.05)
        assert rel < 5e-2
    mc.close()


def test_fit_step_equals_loss_gradient_and_torch_adam():
    """One fused step in FP64 mode: the returned loss is the oracle's, and the parameter
    update equals torch.optim.Adam (CPU) fed with the oracle's gradient."""
    torch = need_gpu()
    from paper_2604_08250_amd.fit import Fitter
    params = _params()
    model = oracle.MLP(1, 128, params)
    L, B = 4, 3
    cells = (L, L, L)
    snaps = synth.snapshots(B, L, seed=44)
    _, ce = _ce()
    labels = np.array([oracle.ce_total(cells, ce, s) for s in snaps])
    mc = _ctx("fp64", params)
    p = torch.from_numpy(params).cuda()
    fit = Fitter(mc, p, lr=1e-3)
    loss = fit.step(torch.from_numpy(snaps).cuda(), torch.from_numpy(labels).cuda(), L)
    l_or, _, g_or = oracle.fit_loss_grad(cells, model, snaps, labels)
    assert loss == pytest.approx(l_or, rel=1e-10)
    ref = torch.from_numpy(params.copy()).requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    ref.grad = torch.from_numpy(g_or.astype(np.float32))
    opt.step()
    got = p.cpu().numpy()
    want = ref.detach().numpy()
    # first Adam step moves every parameter by about lr; FP32 rounding of the update
    assert np.max(np.abs(got - want)) < 1e-6
    assert np.max(np.abs(got - params)) > 5e-4
    mc.close()


def test_bf16_fit_reduces_loss():
    """Fit in BF16 on 64 snapshots of 8^3 cells labelled by the CE: the per-atom loss falls."""
    torch = need_gpu()
    from paper_2604_08250_amd.fit import Fitter, ce_energy
    p_ce, _ = _ce()
    params = synth.mlp_params(108, 128, seed=12, scale=0.5)
    mc = _ctx("bf16", params)
    L, B = 8, 64
    snaps = torch.from_numpy(synth.snapshots(B, L, seed=45)).cuda()
    labels = ce_energy(mc, p_ce, snaps, L)
    p = torch.from_numpy(params).cuda()
    # the step's loss comes from the energies its backward pass sums; they must agree with the
    # forward kernel's
    from paper_2604_08250_amd._lib import smc_energy_fwd
    S = torch.empty(B, dtype=torch.float64, device="cuda")
    smc_energy_fwd(mc.ctx, snaps.data_ptr(), B, L, p.data_ptr(), S.data_ptr())
    N = 2 * L ** 3
    loss_fwd = float((((S - labels) / N) ** 2).mean())
    fit = Fitter(mc, p, lr=3e-3)
    losses = [fit.step(snaps, labels, L) for _ in range(60)]
    _banner(f"bf16 fit: loss {losses[0]:.4e} (forward kernel {loss_fwd:.4e}) -> {losses[-1]:.4e}")
    assert losses[0] == pytest.approx(loss_fwd, rel=1e-4)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.25 * losses[0]
    mc.close()


def test_c5_full_batch_sampled():
    """The full fit batch (1,024 snapshots of 16^3 cells, 8.4 M rows) in the launch shape the
    benchmark times: energies of sampled snapshots against the oracle, and the gradient of
    two sampled snapshots (upstream gradient zero elsewhere) against the oracle's."""
    torch = need_gpu()
    from paper_2604_08250_amd._lib import smc_energy_bwd, smc_energy_fwd
    params = synth.mlp_params(108, 128)
    model = oracle.MLP(1, 128, params)
    L, B = 16, 1024
    cells = (L, L, L)
    snaps = synth.snapshots(B, L, seed=synth.SEED_LATTICE + 100)
    mc = _ctx("bf16", params)
    d_snaps = torch.from_numpy(snaps).cuda()
    d_p = torch.from_numpy(params).cuda()
    S = torch.empty(B, dtype=torch.float64, device="cuda")
    _banner("c5 full batch forward")
    smc_energy_fwd(mc.ctx, d_snaps.data_ptr(), B, L, d_p.data_ptr(), S.data_ptr())
    S = S.cpu().numpy()
    picks = [0, 517, 1023]
    S_or = oracle.snapshot_energies(cells, model, snaps[picks])
    per_atom = np.abs(S[picks] - S_or) / snaps.shape[1]
    _banner(f"c5 sampled energies: per-atom error {per_atom.max():.2e} eV")
    assert np.all(per_atom < 1e-3)
    gE = np.zeros(B)
    gE[3], gE[700] = 1.0, -2.0
    grad = torch.empty_like(d_p)
    smc_energy_bwd(mc.ctx, d_snaps.data_ptr(), B, L, d_p.data_ptr(), torch.from_numpy(gE).cuda().data_ptr(),
                   grad.data_ptr())
    grad = grad.cpu().numpy().astype(np.float64)
    g_or = oracle.energy_grad(cells, model, snaps[[3, 700]], gE[[3, 700]])
    r = np.linalg.norm(grad - g_or) / np.linalg.norm(g_or)
    _banner(f"c5 sampled gradient rel err vs fp64 {r:.2e}")
    assert r < 5e-2
    mc.close()


def test_mc_snapshots():
    """Snapshot chains by swap MC on the CE pair part (the fit's training snapshots): the shape
    and each chain's composition are kept; each snapshot equals the oracle's sweeps of its
    chain with the qSRO blob that carries the CE pairs; the same seed gives the same snapshots;
    and from one start, the chain at 300 K ends lower in CE pair energy than the one at 3000 K."""
    torch = need_gpu()
    from paper_2604_08250_amd.fit import ce_pair_qsro, sample_snapshots
    L, B = 6, 4
    N = 2 * L ** 3
    cells = (L, L, L)
    start = synth.snapshots(B, L, seed=50)
    temps = synth.snapshot_temperatures(B)
    pair = synth.ce_params()["pair"]
    _banner("mc snapshots")
    out = sample_snapshots(start, L, temps, pair, burn_in=3, n_per_chain=2, gap=2, seed=13)
    assert tuple(out.shape) == (2 * B, N) and out.dtype == torch.uint8
    got = out.cpu().numpy()
    for k in range(2):
        for b in range(B):
            assert np.array_equal(np.bincount(got[k * B + b], minlength=4), np.bincount(start[b], minlength=4))
    model = oracle.QSRO(ce_pair_qsro(pair))
    for b in range(B):
        ref = start[b].copy()
        for t in range(3):
            oracle.sweep(cells, model, ref, temps[b], 13, b, t, nthreads=8)
        assert np.array_equal(got[b], ref), f"chain {b} after burn-in"
        for t in range(3, 5):
            oracle.sweep(cells, model, ref, temps[b], 13, b, t, nthreads=8)
        assert np.array_equal(got[B + b], ref), f"chain {b} snapshot 1"
    again = sample_snapshots(start, L, temps, pair, burn_in=3, n_per_chain=2, gap=2, seed=13).cpu().numpy()
    assert np.array_equal(again, got)
    # temperature: one start, 300 K against 3000 K
    two = np.stack([start[0], start[0]])
    cold_hot = sample_snapshots(two, L, [300.0, 3000.0], pair, burn_in=40, seed=14).cpu().numpy()
    ce = oracle.CEModel(4, pair, np.zeros((0, 6)), np.zeros((0, 3)), np.zeros(0))
    e = [oracle.ce_total(cells, ce, s) / N for s in cold_hot]
    _banner(f"CE pair energy per atom after 40 sweeps: 300 K {e[0]:.5f}, 3000 K {e[1]:.5f}")
    assert e[0] < e[1]
