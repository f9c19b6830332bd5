"""Full-size parity: the benchmark workload (921 x 301 layered-faulted model,
64 shots, 461 receivers, 4000 steps, K = 50) in the benchmark's launch
configuration (64-shot plans, batches of 16), against oracle fixtures for one
sampled shot (tests/golden/make_full_size.py), plus identities that hold at
any size.

Sampling inside the 64-shot launch: the migration of a residual that is zero
for every shot but the sampled one equals that shot's migration.  The
Gauss-Newton product sums over shots, so its per-shot fixture is compared
with a one-shot plan, and the 64-shot product is checked through the
dot-product test, symmetry and additivity over shot subsets.

Tolerances: 4000 FP32 leapfrog steps accumulate more rounding than the 500 of
the small case; measured errors are printed.  The forward data meet the 1e-5
target per output; the Hessian products are bounded at 1e-5 (2.5-4x above
the measured values), the Born data at about 2x their measured error, and
the images at the 1e-4 target.
"""
import os
import sys

import numpy as np
import pytest

from paper_2507_10804_amd import synth
from tests._cases import rel

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import torch
    from paper_2507_10804_amd import fwi
    g, m_true, m_eval = synth.config_layered()
    plan = fwi.Plan(g)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device="cuda")
    return dict(torch=torch, fwi=fwi, g=g, m_true=m_true, m_eval=m_eval, plan=plan, f32=f32)


def host(x):
    return x.detach().double().cpu().numpy()


def test_full_forward_sampled_shot(full):
    say("entry: fwi_forward 921x301, 64 shots, nt=4000 (sampled shot vs oracle)")
    gold = np.load(os.path.join(GOLD, "full_size_forward.npz"))
    s, rs, ts = int(gold["shot"]), int(gold["rec_stride"]), int(gold["t_stride"])
    d = full["plan"].forward(full["f32"](full["m_true"]))
    got = host(d[s, ::ts, ::rs])
    e = rel(got, gold["d"])
    say(f"  rel-L2 forward data (shot {s}) = {e:.3e}")
    assert e < 1e-5
    assert full["plan"].status() == 0


def test_full_adjoint_sampled_shot(full):
    say("entry: fwi_adjoint 921x301, 64 shots, B=16 (sampled shot vs oracle)")
    torch, g = full["torch"], full["g"]
    gold = np.load(os.path.join(GOLD, "full_size_adjoint.npz"))
    s = int(gold["shot"])
    # every batch member holds the same residual on the sampled shot with
    # its own scale (b+1)/16, so a mix-up of members inside a workgroup fails
    r = np.zeros((16, g.ns, g.nt, g.nr), np.float32)
    r0 = synth.residual_noise((1, g.nt, g.nr), seed=int(gold["r_seed"]))[0]
    for b in range(16):
        r[b, s] = (b + 1) / 16 * r0
    out = host(full["plan"].adjoint(full["f32"](full["m_eval"]), full["f32"](r)))
    del r
    e = [rel(out[b], (b + 1) / 16 * gold["g"]) for b in range(16)]
    say(f"  rel-L2 migration (shot {s}): member 15 {e[15]:.3e}, max over members {max(e):.3e}")
    assert max(e) < 1e-4


def test_full_gn_hvp_sampled_shot(full):
    say("entry: fwi_gn_hvp 921x301, one sampled shot, nt=4000")
    fwi = full["fwi"]
    gold = np.load(os.path.join(GOLD, "full_size_hvp.npz"))
    s = int(gold["shot"])
    g1 = full["g"].with_shots([s])
    plan1 = fwi.Plan(g1)
    v = synth.smooth_random((g1.nz, g1.nx), seed=int(gold["v_seed"]), sigma=5.0)
    hv = host(plan1.gn_hvp(full["f32"](full["m_eval"]), full["f32"](v)))
    e = rel(hv, gold["hv"])
    say(f"  rel-L2 GN Hv (shot {s}) = {e:.3e}")
    assert e < 1e-5


def test_full_born_sampled_shot(full):
    """Born data at full size in the benchmark's batch of 16, every member a
    distinct multiple of the fixture's vector, sampled on one shot against
    the oracle (target 1e-5 per output; bound about twice the measured
    1.7e-5)."""
    say("entry: fwi_born 921x301, 64 shots, B=16 (sampled shot vs oracle)")
    g = full["g"]
    full["plan"].release_workspaces()
    gold = np.load(os.path.join(GOLD, "full_size_born.npz"))
    s, rs, ts = int(gold["shot"]), int(gold["rec_stride"]), int(gold["t_stride"])
    v = synth.smooth_random((g.nz, g.nx), seed=int(gold["v_seed"]), sigma=5.0)
    V = np.stack([(b + 1) / 16 * v for b in range(16)])
    dd = full["plan"].born(full["f32"](full["m_eval"]), full["f32"](V))
    got = host(dd[:, s, ::ts, ::rs])
    del dd
    full["plan"].release_workspaces()
    e = [rel(got[b], (b + 1) / 16 * gold["dd"]) for b in range(16)]
    say(f"  rel-L2 Born data (shot {s}): member 0 {e[0]:.3e}, max over members {max(e):.3e}")
    assert max(e) < 3.5e-5


def test_full_fused_grad_hvp_vs_oracle(full):
    """The benchmark's call, fwi_misfit_grad_hvp with B = 16, on the sampled
    shot's plan: 17 adjoint right-hand sides in workgroups of two (the last
    one holding a single vector), in the benchmark's launch configuration.
    Members are distinct multiples (b+1)/16 of the fixture's vector; Phi, the
    gradient and all 16 products are compared with the oracle.  The observed
    data come from the GPU forward map of the true model (FP32, 4.5e-6 from
    the oracle's), whose error the residual amplifies by |dobs|/|d - dobs|."""
    say("entry: fwi_misfit_grad_hvp 921x301, one sampled shot, B=16 (vs oracle)")
    fwi, f32 = full["fwi"], full["f32"]
    full["plan"].release_workspaces()
    gh = np.load(os.path.join(GOLD, "full_size_hvp.npz"))
    gg = np.load(os.path.join(GOLD, "full_size_grad.npz"))
    s = int(gh["shot"])
    assert int(gg["shot"]) == s
    g1 = full["g"].with_shots([s])
    plan1 = fwi.Plan(g1)
    v = synth.smooth_random((g1.nz, g1.nx), seed=int(gh["v_seed"]), sigma=5.0)
    V = np.stack([(b + 1) / 16 * v for b in range(16)])
    dobs = plan1.forward(f32(full["m_true"]))
    phi, grad, hv = plan1.misfit_grad_hvp(f32(full["m_eval"]), dobs, f32(V))
    hv, grad, phi = host(hv), host(grad), float(phi)
    amp = float(dobs.double().norm()) / np.sqrt(2 * float(gg["phi"]))
    assert plan1.status() == 0
    eh = [rel(hv[b], (b + 1) / 16 * gh["hv"]) for b in range(16)]
    eg = rel(grad, gg["grad"])
    ep = abs(phi - float(gg["phi"])) / float(gg["phi"])
    say(f"  Phi rel {ep:.2e}; gradient {eg:.3e} (residual amplification {amp:.1f}); "
        f"H v member 0 {eh[0]:.3e}, member 15 (the lone last group) {eh[15]:.3e}, "
        f"max {max(eh):.3e}")
    assert max(eh) < 1e-5
    assert eg < max(1e-4, 3 * 1.3e-5 * amp)
    assert ep < max(1e-4, 2 * 1.3e-5 * amp)


def test_full_probe_batch_one_shot_vs_oracle(full):
    """A batched-probing launch: 64 products at once through a ProbeSession
    (graph-captured time loops) on the sampled shot's plan, holding the two
    probe families -- an impulse comb with deltas every 40 cells and a
    Rademacher field smoothed over 5 cells -- among 62 other probes; both
    against the oracle, and the comb again, halved, in the last slot."""
    from paper_2507_10804_amd import probing
    say("entry: ProbeSession B=64 at 921x301, one sampled shot (vs oracle)")
    fwi, f32, g = full["fwi"], full["f32"], full["g"]
    full["plan"].release_workspaces()
    gold = np.load(os.path.join(GOLD, "full_size_probe.npz"))
    s = int(gold["shot"])
    combs = synth.impulse_combs(g.nz, g.nx, count=64, spacing=40, seed=int(gold["comb_seed"]))
    rads = synth.rademacher_smoothed(g.nz, g.nx, seeds=range(int(gold["rad_seed"]),
                                                            int(gold["rad_seed"]) + 31))
    V = np.concatenate([combs[:1], rads[:1], combs[1:32], rads[1:31], 0.5 * combs[:1]])
    assert V.shape[0] == 64
    plan1 = fwi.Plan(g.with_shots([s]))
    sess = probing.ProbeSession(plan1, f32(full["m_eval"]), 64)
    hv = host(sess.run(f32(V)))
    assert plan1.status() == 0
    ec, er = rel(hv[0], gold["hv_comb"]), rel(hv[1], gold["hv_rad"])
    eh = rel(hv[63], 0.5 * gold["hv_comb"])
    say(f"  rel-L2 comb {ec:.3e}, smoothed Rademacher {er:.3e}, halved comb (slot 63) {eh:.3e}")
    assert max(ec, er, eh) < 1e-5


def test_full_probe_batch_64_shots(full):
    """Launch A of the probing workload as timed: 64 impulse combs (deltas
    every 40 cells) on all 64 shots in one graph-captured B = 64 launch.
    Shots are summed in groups here, so the per-shot fixtures do not apply;
    checked instead: Hessian symmetry and positivity between members, and a
    member against a separate single-vector product (another launch shape
    and shot grouping)."""
    from paper_2507_10804_amd import probing
    say("entry: ProbeSession B=64 at 921x301, 64 shots (combs; identities)")
    f32, g, plan = full["f32"], full["g"], full["plan"]
    plan.release_workspaces()
    combs = synth.impulse_combs(g.nz, g.nx, count=64, spacing=40, seed=100)
    m = f32(full["m_eval"])
    sess = probing.ProbeSession(plan, m, 64)
    hv = host(sess.run(f32(combs)))
    assert plan.status() == 0
    # combs with different offsets barely couple, so the error is measured
    # against the Cauchy-Schwarz scale sqrt(<a, H a> <b, H b>)
    sym = []
    for a, b in [(0, 1), (5, 40), (62, 63)]:
        x, y = np.vdot(combs[a], hv[b]), np.vdot(hv[a], combs[b])
        scale = np.sqrt(np.vdot(combs[a], hv[a]) * np.vdot(combs[b], hv[b]))
        sym.append(abs(x - y) / scale)
    say(f"  symmetry max rel {max(sym):.2e}")
    assert max(sym) < 1e-5
    assert all(np.vdot(combs[b], hv[b]) > 0 for b in range(64))
    del sess
    plan.release_workspaces()
    h5 = host(plan.gn_hvp(m, f32(combs[5])))
    e = rel(hv[5], h5)
    say(f"  member 5 vs single-vector call {e:.2e}")
    assert e < 1e-6
    plan.release_workspaces()


def _band_limited(torch, shape, f0, dt, seed):
    """N(0,1) traces filtered in time to the Ricker spectrum of peak f0: a
    residual with the band of real data."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(shape, generator=gen, device="cuda", dtype=torch.float32)
    nt = shape[-2]
    f = torch.fft.rfftfreq(nt, d=dt, device="cuda")
    spec = (f / f0) ** 2 * torch.exp(-((f / f0) ** 2))
    X = torch.fft.rfft(x, dim=-2) * spec[:, None].to(torch.complex64)
    return torch.fft.irfft(X, n=nt, dim=-2).contiguous()


def test_full_dot_product_and_symmetry(full):
    """Batches of 16 at full size, as the benchmark launches them.

    For a random residual r, <J v, r> keeps only the part of r that looks
    like data and cancels by a factor |Jv||r| / |<Jv, r>| of 10^3..10^4 here,
    so the plain relative error of the dot test measures that cancellation
    more than the adjoint.  The test therefore bounds the normalised error
    |<Jv,r> - <v,J^T r>| / (|Jv||r|) for white and band-limited random r, and
    the plain relative error for a data-like residual r = J (v_b + v_{b+1})."""
    say("entry: fwi_born + fwi_adjoint + fwi_gn_hvp B=16 at full size")
    torch, g, plan = full["torch"], full["g"], full["plan"]
    m = full["f32"](full["m_eval"])
    vs = synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, 17))
    V = full["f32"](vs)
    jv = plan.born(m, V)
    for kind in ("data-like", "band", "white"):
        if kind == "band":
            r = _band_limited(torch, tuple(jv.shape), g.f0, g.dt, seed=3)
        elif kind == "white":
            r = torch.empty_like(jv).normal_(
                generator=torch.Generator(device="cuda").manual_seed(3))
        else:
            r = jv + jv.roll(-1, dims=0)
        jtr = plan.adjoint(m, r)
        lhs = (jv.double() * r.double()).sum(dim=(1, 2, 3)).cpu().numpy()
        rhs = (V.double() * jtr.double()).sum(dim=(1, 2)).cpu().numpy()
        scale = (jv.double().flatten(1).norm(dim=1) * r.double().flatten(1).norm(dim=1))
        scale = scale.cpu().numpy()
        err = np.abs(lhs - rhs) / np.abs(lhs)
        nerr = np.abs(lhs - rhs) / scale
        say(f"  dot test ({kind} r): max rel {err.max():.3e}, normalised {nerr.max():.3e}, "
            f"cancellation factor {np.min(scale / np.abs(lhs)):.0f}.."
            f"{np.max(scale / np.abs(lhs)):.0f}")
        assert nerr.max() < 1e-7
        if kind == "data-like":
            assert err.max() < 1e-5
        del r, jtr
    del jv
    hv = host(plan.gn_hvp(m, V))
    sym = []
    for a, b in [(0, 1), (2, 7), (5, 15)]:
        x, y = np.vdot(vs[a], hv[b]), np.vdot(hv[a], vs[b])
        sym.append(abs(x - y) / abs(x))
    say(f"  symmetry max rel = {max(sym):.3e}")
    assert max(sym) < 1e-5
    assert all(np.vdot(vs[b], hv[b]) > 0 for b in range(16))


def test_full_shot_additivity(full):
    """H over 64 shots equals the sum over two 32-shot halves (shots are
    independent; the grouping of the FP64 image sum differs)."""
    say("entry: fwi_gn_hvp 64 shots vs 2 x 32 shots")
    fwi, g, plan = full["fwi"], full["g"], full["plan"]
    m = full["f32"](full["m_eval"])
    v = full["f32"](synth.smooth_random((g.nz, g.nx), seed=21, sigma=5.0))
    h64 = host(plan.gn_hvp(m, v))
    plan.release_workspaces()
    ha = host(fwi.Plan(g.with_shots(range(0, 32))).gn_hvp(m, v))
    hb = host(fwi.Plan(g.with_shots(range(32, 64))).gn_hvp(m, v))
    e = rel(ha + hb, h64)
    say(f"  rel-L2 additivity = {e:.3e}")
    assert e < 1e-6


def test_full_fused_grad_hvp(full):
    """The benchmark's call: misfit, gradient and 16 products in one pass at
    full size, against the separate calls in the same launch configuration."""
    say("entry: fwi_misfit_grad_hvp B=16 at full size vs fwi_misfit_grad + fwi_gn_hvp")
    torch, g, plan, f32 = full["torch"], full["g"], full["plan"], full["f32"]
    plan.release_workspaces()
    m = f32(full["m_eval"])
    dobs = plan.forward(f32(full["m_true"]))
    V = f32(synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, 17)))
    phi, grad, hv = plan.misfit_grad_hvp(m, dobs, V)
    hv = host(hv)
    grad = host(grad)
    phi = float(phi)
    plan.release_workspaces()
    phi_s, grad_s = plan.misfit_grad(m, dobs)
    eg = rel(grad, host(grad_s))
    del grad_s
    plan.release_workspaces()
    eh = rel(hv, host(plan.gn_hvp(m, V)))
    say(f"  Phi {phi:.6e} vs {float(phi_s):.6e}; gradient {eg:.2e}; H v {eh:.2e}")
    assert phi == float(phi_s)
    assert eg < 1e-6 and eh < 1e-6
    plan.release_workspaces()


def test_full_autograd(full):
    """The differentiation layer at full size: the backward of FwiForward for
    a residual on the sampled shot equals that shot's oracle migration, and
    the misfit gradient agrees with a central difference of the misfit
    (h = 1e-3 relative; FP32 data bound the agreement to ~1e-3)."""
    from paper_2507_10804_amd import autograd as ag
    say("entry: autograd FwiForward / Misfit at 921x301, 64 shots, nt=4000")
    torch, g, plan, f32 = full["torch"], full["g"], full["plan"], full["f32"]
    plan.release_workspaces()
    gold = np.load(os.path.join(GOLD, "full_size_adjoint.npz"))
    s = int(gold["shot"])
    r = np.zeros((g.ns, g.nt, g.nr), np.float32)
    r[s] = synth.residual_noise((1, g.nt, g.nr), seed=int(gold["r_seed"]))[0]
    m = f32(full["m_eval"]).requires_grad_(True)
    d = ag.forward(m, plan)
    (gm,) = torch.autograd.grad(d, m, grad_outputs=f32(r))
    e = rel(host(gm), gold["g"])
    say(f"  rel-L2 autograd backward (shot {s}) = {e:.3e}")
    assert e < 1e-4
    del d, gm
    dobs = plan.forward(f32(full["m_true"]))
    m0 = full["m_eval"]
    v = synth.smooth_random((g.nz, g.nx), seed=1, sigma=5.0)
    mm = f32(m0).requires_grad_(True)
    ag.misfit(mm, dobs, plan).backward()
    dirv = float(np.vdot(host(mm.grad), v))
    h = 1e-3 * np.abs(m0).max() / np.abs(v).max()
    fp = float(plan.misfit(f32(m0 + h * v), dobs))
    fm = float(plan.misfit(f32(m0 - h * v), dobs))
    fd = (fp - fm) / (2 * h)
    say(f"  FD {fd:.6e} vs <grad, v> {dirv:.6e} (rel {abs(fd - dirv) / abs(dirv):.2e})")
    assert fd == pytest.approx(dirv, rel=2e-3)
