"""GPU tests of the layers above the C ABI: the autograd Function (checked
against the FP64 oracle and central finite differences), the fused misfit,
the checkpoint-resuming adjoint and the graph-captured probing session."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_10804_amd import synth
from tests._cases import rel, tiny

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def dev(torch, x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda")


def host(x):
    return x.detach().double().cpu().numpy()


@pytest.fixture(scope="module")
def case(torch):
    from paper_2507_10804_amd import fwi
    g, m_true, _ = synth.config_small()
    m = 1.05 * m_true  # residual comparable to the data: well conditioned
    dobs = oracle.forward(g, m_true)
    v = synth.smooth_random((g.nz, g.nx), seed=1, sigma=5.0)
    return dict(g=g, m=m, dobs=dobs, v=v, plan=fwi.Plan(g))


def test_autograd_gradient_vs_oracle(torch, case):
    from paper_2507_10804_amd import autograd as ag
    say("entry: FwiForward backward (adjoint_resume) small")
    g, plan = case["g"], case["plan"]
    m = dev(torch, case["m"]).requires_grad_(True)
    dobs = dev(torch, case["dobs"])
    d = ag.forward(m, plan)
    phi = 0.5 * ((d.double() - dobs.double()) ** 2).sum()
    phi.backward()
    phi_o, grad_o = oracle.misfit_grad(g, case["m"], case["dobs"])
    assert float(phi) == pytest.approx(phi_o, rel=1e-4)
    assert rel(host(m.grad), grad_o) < 1e-4
    # the fused misfit Function gives the same gradient
    m2 = dev(torch, case["m"]).requires_grad_(True)
    ag.misfit(m2, dobs, plan).backward()
    assert rel(host(m2.grad), grad_o) < 1e-4


def test_backward_repeatable(torch, case):
    from paper_2507_10804_amd import autograd as ag
    say("entry: repeated backward on one forward")
    plan = case["plan"]
    m = dev(torch, case["m"]).requires_grad_(True)
    d = ag.forward(m, plan)
    r = dev(torch, synth.residual_noise(tuple(d.shape), seed=4))
    (g1,) = torch.autograd.grad(d, m, grad_outputs=r, retain_graph=True)
    (g2,) = torch.autograd.grad(d, m, grad_outputs=r)
    assert torch.equal(g1, g2)
    assert rel(host(g1), host(plan.adjoint(m.detach(), r))) < 1e-6


def test_autograd_finite_difference(torch, case):
    """Central difference of Phi along v, h = 1e-3 relative, against
    <grad, v>: FP32 data limit the agreement to ~1e-3."""
    from paper_2507_10804_amd import autograd as ag
    say("entry: misfit finite difference small")
    plan, v = case["plan"], case["v"]
    m0 = case["m"]
    dobs = dev(torch, case["dobs"])
    m = dev(torch, m0).requires_grad_(True)
    ag.misfit(m, dobs, plan).backward()
    dirv = float(np.vdot(host(m.grad), v))
    h = 1e-3 * np.abs(m0).max() / np.abs(v).max()
    fp = float(plan.misfit(dev(torch, m0 + h * v), dobs))
    fm = float(plan.misfit(dev(torch, m0 - h * v), dobs))
    fd = (fp - fm) / (2 * h)
    say(f"  FD {fd:.6e} vs <grad, v> {dirv:.6e}")
    assert fd == pytest.approx(dirv, rel=2e-3)


def test_jvp_and_gn_hvp_autograd(torch, case):
    from paper_2507_10804_amd import autograd as ag
    say("entry: forward-mode jvp and vjp-of-jvp small")
    g, plan, m, v = case["g"], case["plan"], case["m"], case["v"]
    jv = ag.born_jvp(dev(torch, m), dev(torch, v), plan)
    assert rel(host(jv), oracle.born(g, m, v)) < 1e-5
    hv = ag.gn_hvp_autograd(dev(torch, m), dev(torch, v), plan)
    ho = oracle.gn_hvp(g, m, v)
    assert rel(host(hv), ho) < 1e-4
    assert rel(host(hv), host(ag.gn_hvp(dev(torch, m), dev(torch, v), plan))) < 1e-5


def test_misfit_only(torch, case):
    say("entry: fwi_misfit small")
    g, plan = case["g"], case["plan"]
    phi = float(plan.misfit(dev(torch, case["m"]), dev(torch, case["dobs"])))
    phi_o, _ = oracle.misfit_grad(g, case["m"], case["dobs"])
    assert phi == pytest.approx(phi_o, rel=1e-4)


def test_probe_session_graph_replays(torch):
    """The captured call replayed several times, with eager work and
    synchronisations in between, matches the eager call every time."""
    from paper_2507_10804_amd import fwi, probing
    say("entry: ProbeSession graph capture tiny, B=4")
    g, m = tiny(nt=160)
    plan = fwi.Plan(g)
    combs = synth.impulse_combs(g.nz, g.nx, count=4, spacing=12, seed=100)
    rad = synth.rademacher_smoothed(g.nz, g.nx, seeds=[200, 201, 202, 203], sigma=2.0)
    sess = probing.ProbeSession(plan, dev(torch, m), batch=4, use_graph=True)
    eager = fwi.Plan(g)
    for rep, batch in enumerate([combs, rad, combs, rad[:3]]):
        out = host(sess.run(dev(torch, batch)))
        ref = host(eager.gn_hvp(dev(torch, m), dev(torch, batch)))
        torch.cuda.synchronize()
        if batch.shape[0] == 4:
            assert np.array_equal(out, ref), f"replay {rep} differs from eager"
        else:  # zero-padded batch: another shot grouping in the adjoint
            assert rel(out, ref) < 1e-6
        _ = (dev(torch, batch) * 2).sum().item()  # unrelated eager work in between
    assert rel(host(sess.run(dev(torch, combs))), oracle.gn_hvp(g, m, combs)) < 1e-4


def test_probe_session_history_mode(torch):
    """A probe session on a plan that keeps the whole forward history
    (ckpt_every = 0): the captured call stores every w^n in the forward sweep
    and recomputes nothing, and its replays equal the eager call and the
    checkpointed plan's products bit for bit (nt - 1 odd: the adjoint pairs
    its steps alike in both modes)."""
    from paper_2507_10804_amd import fwi, probing
    say("entry: ProbeSession graph capture tiny, history mode, B=4")
    g, m = tiny(nt=160)
    rad = synth.rademacher_smoothed(g.nz, g.nx, seeds=[300, 301, 302, 303], sigma=2.0)
    ckpt = host(fwi.Plan(g).gn_hvp(dev(torch, m), dev(torch, rad)))
    g.ckpt_every = 0
    plan = fwi.Plan(g)
    assert plan.K == g.nt - 1 and plan.history
    sess = probing.ProbeSession(plan, dev(torch, m), batch=4, use_graph=True)
    for rep in range(3):
        out = host(sess.run(dev(torch, rad)))
        torch.cuda.synchronize()
        assert np.array_equal(out, ckpt), f"replay {rep} differs from the checkpointed plan"
        _ = (dev(torch, rad) * 2).sum().item()
    assert np.array_equal(host(plan.gn_hvp(dev(torch, m), dev(torch, rad))), ckpt)
    assert plan.status() == 0


def test_probe_session_survives_workspace_release(torch):
    """A session keeps its own workspace: after the plan drops its cached
    workspaces and the memory is handed to another tensor, replays still
    give the same result and leave that tensor untouched."""
    from paper_2507_10804_amd import fwi, probing
    say("entry: ProbeSession replay after Plan.release_workspaces, tiny, B=2")
    g, m = tiny(nt=120)
    plan = fwi.Plan(g)
    v = synth.smooth_random_batch(g.nz, g.nx, seeds=[11, 12], sigma=2.0)
    sess = probing.ProbeSession(plan, dev(torch, m), batch=2, use_graph=True)
    first = host(sess.run(dev(torch, v))).copy()
    plan.workspace(fwi.FWI_OP_GN_HVP, 2)  # a cached workspace of the same size
    nbytes = plan.workspace_bytes(fwi.FWI_OP_GN_HVP, 2)
    plan.release_workspaces()
    torch.cuda.synchronize()
    sentinel = torch.full((nbytes // 4,), 7.25, dtype=torch.float32, device="cuda")
    again = host(sess.run(dev(torch, v)))
    torch.cuda.synchronize()
    assert np.array_equal(first, again)
    assert bool((sentinel == 7.25).all())
