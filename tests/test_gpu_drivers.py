"""L-BFGS and gpCN drivers on the GPU against the FP64 oracle
(oracle/drivers.py), through the C ABI of include/fwi_opt.h and the plan,
prior and low-rank entry points.

* dot products and updates against NumPy; the two-loop recursion against
  the oracle's for 5 stored pairs (rel 1e-6: FP64 accumulation of FP32
  vectors);
* three L-BFGS iterations with the prior R^-1 as initial inverse Hessian on
  the 128 x 128 / 4-shot wave problem, started (and prior-centred) at a
  model 5 % faster than the truth: there the residual is comparable to the
  data (|d| / |d - d_obs| = 3.6), so FP32 wave solves give the gradient to
  ~1e-4 (at the smoothed start the ratio is 754 and the gradient agrees only
  to ~1e-2, enough to flip a line-search decision).  Identical step lengths
  and backtracking counts (the oracle's Armijo tests clear their thresholds
  by >= 16 % of Phi; a trial with a non-positive velocity is rejected on
  both sides), Phi within 1e-3, the iterate's update within 1e-3;
* five gpCN steps (beta = 0.1) with an R-orthonormal rank-6 Laplace
  approximation from given pairs: identical accept/reject decisions (the
  oracle's acceptance probabilities clear the uniforms by >= 0.08), Delta
  within 1e-3 absolute, final state within 1e-4.
"""
import sys

import numpy as np
import pytest

from oracle import drivers as Dr
from oracle import lowrank as LR
from paper_2507_10804_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(x):
    return x.detach().double().cpu().numpy()


def r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_vector_ops_and_two_loop():
    import ctypes

    import torch
    from paper_2507_10804_amd import drivers as D

    n = 12345
    rng = np.random.default_rng(0)
    say(f"case: fwi_vec_dot/update and fwi_lbfgs_loop1/loop2, n={n}, 5 pairs")
    v = D.Vec(n, torch.device("cuda"))
    x, y = r32(rng.standard_normal(n)), r32(rng.standard_normal(n))
    xd, yd = dev(torch, x), dev(torch, y)
    assert v.dot(xd, yd) == pytest.approx(float(x @ y), rel=1e-12)
    v.update(0.5, xd, -2.0, yd)
    assert np.allclose(host(yd), r32(0.5 * x - 2.0 * y), rtol=1e-6, atol=1e-6)
    # two-loop recursion with gamma from the newest pair
    m = 5
    S = [r32(rng.standard_normal(n)) for _ in range(m)]
    Y = [r32(s * rng.uniform(0.5, 2.0, n) + 0.1 * rng.standard_normal(n)) for s in S]
    g = r32(rng.standard_normal(n))
    slots = [3, 0, 4, 1, 2]  # oldest .. newest, deliberately out of order
    Sd = torch.zeros((6, n), dtype=torch.float32, device="cuda")
    Yd = torch.zeros_like(Sd)
    rho = torch.zeros(6, dtype=torch.float64, device="cuda")
    alpha = torch.zeros(6, dtype=torch.float64, device="cuda")
    gam = torch.ones(1, dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    for k, sl in enumerate(slots):
        Sd[sl] = dev(torch, S[k])
        Yd[sl] = dev(torch, Y[k])
        D.fwi._check(v.lib.fwi_lbfgs_pair(n, p(Sd[sl]), p(Yd[sl]), p(rho[sl:]), p(gam), p(v.ws),
                                          v.nws, v.st()))
    order = list(reversed(slots))
    arr = (ctypes.c_int * m)(*order)
    q = dev(torch, g)
    D.fwi._check(v.lib.fwi_lbfgs_loop1(n, m, arr, p(Sd), p(Yd), p(rho), p(q), p(alpha), p(v.ws),
                                       v.nws, v.st()))
    r = torch.empty_like(q)
    v.update(1.0, q, 0.0, r, ad=gam)
    D.fwi._check(v.lib.fwi_lbfgs_loop2(n, m, arr, p(Sd), p(Yd), p(rho), p(alpha), p(r), p(v.ws),
                                       v.nws, v.st()))
    gam_o = float(S[-1] @ Y[-1] / (Y[-1] @ Y[-1]))
    ref = Dr.two_loop(g, S, Y, lambda qq: gam_o * qq)
    e = np.linalg.norm(host(r) - ref) / np.linalg.norm(ref)
    say(f"  gamma {float(gam.item()):.12g} (oracle {gam_o:.12g}); two-loop rel-L2 {e:.2e}")
    assert float(gam.item()) == pytest.approx(gam_o, rel=1e-12)
    assert e < 1e-6


def _wave_problem(start="smoothed"):
    import oracle

    g, m_true, m_eval = synth.config_small()
    dobs = r32(oracle.forward(g, m_true))
    P = synth.matern_prior(g.nz, g.nx, g.dx, 300.0, 100.0)
    m0 = m_eval if start == "smoothed" else 1.05 * m_true
    return g, dobs, P, r32(m0)


def test_lbfgs_matches_oracle():
    import torch
    from paper_2507_10804_amd import drivers as D
    from paper_2507_10804_amd import fwi
    from paper_2507_10804_amd import lowrank as glr

    g, dobs, P, m0 = _wave_problem("faster")
    say(f"case: L-BFGS, H0 = R^-1, 3 iterations, 128x128, 4 shots, nt={g.nt}, 5% faster start")
    pr = LR.Prior(P)
    ref = Dr.lbfgs(lambda m: Dr.objective(g, pr, m0, dobs, m), m0, 3, h0=pr.solve)
    plan = fwi.Plan(g)
    gp = glr.Prior(P)
    post = D.Posterior(plan, gp, dev(torch, m0), dev(torch, dobs))
    opt = D.Lbfgs(post, dev(torch, m0), h0=lambda q: gp.apply(glr.PRIOR_RINV, q))
    hist = opt.run(3)
    say(f"  t {hist['t']} (oracle {ref['t']}), backtracks {hist['backtracks']} "
        f"(oracle {ref['backtracks']})")
    say(f"  Phi {['%.8e' % f for f in hist['phi']]}")
    say(f"  oracle {['%.8e' % f for f in ref['phi']]}")
    assert hist["t"] == ref["t"] and hist["backtracks"] == ref["backtracks"]
    assert np.allclose(hist["phi"], ref["phi"], rtol=1e-3)
    du, du_o = host(opt.m) - m0, ref["m"][-1] - m0
    e = np.linalg.norm(du - du_o) / np.linalg.norm(du_o)
    say(f"  update rel-L2 {e:.2e}")
    assert e < 1e-3


def test_gpcn_matches_oracle():
    import torch
    from paper_2507_10804_amd import drivers as D
    from paper_2507_10804_amd import fwi
    from paper_2507_10804_amd import lowrank as glr

    g, dobs, P, m0 = _wave_problem()
    pr = LR.Prior(P)
    rng = np.random.default_rng(2)
    r = 6
    X = pr.sqrt_inv(rng.standard_normal((r, P.nz, P.nx))).reshape(r, -1)
    Q, _ = LR.r_orthonormalize(X, pr.apply(X.reshape(r, P.nz, P.nx)).reshape(r, -1))
    V = r32(Q.reshape(r, P.nz, P.nx))
    lam = np.geomspace(5.0, 0.1, r)
    w = r32(rng.standard_normal((5, P.nz, P.nx)))
    u = rng.uniform(size=5)
    beta = 0.1
    say(f"case: gpCN, beta={beta}, 5 steps, rank-{r} Laplace approximation, 128x128")
    phi = lambda m: Dr.objective(g, pr, m0, dobs, m)[0]
    st_o, acc_o, de_o = Dr.gpcn(phi, m0, m0, beta, lambda wk: LR.sample(pr, lam, V, wk),
                                lambda x: LR.hessian_apply(pr, lam, V, x), w, u)
    plan = fwi.Plan(g)
    gp = glr.Prior(P)
    lr = glr.LowRank.from_pairs(gp, torch.as_tensor(lam, device="cuda"), dev(torch, V))
    post = D.Posterior(plan, gp, dev(torch, m0), dev(torch, dobs))
    md = dev(torch, m0)
    st, acc, de = D.gpcn(post, md, md, beta, lr.sample, lr.hessian, dev(torch, w), u)
    say(f"  accepted {acc} (oracle {acc_o}); Delta {['%.5f' % d for d in de]}")
    say(f"  oracle Delta {['%.5f' % d for d in de_o]}")
    assert acc == acc_o
    assert np.allclose(de, de_o, atol=1e-3)
    e = np.linalg.norm(host(st[-1]) - st_o[-1]) / np.linalg.norm(st_o[-1])
    say(f"  final state rel-L2 {e:.2e}")
    assert e < 1e-4


def test_dot_is_reproducible():
    """FP64 dot products with a fixed grid and summation order: bitwise
    identical run to run, at the full model size."""
    import torch
    from paper_2507_10804_amd import drivers as D

    n = 301 * 921
    say(f"case: fwi_vec_dot reproducibility, n={n}")
    v = D.Vec(n, torch.device("cuda"))
    rng = np.random.default_rng(5)
    x, y = dev(torch, rng.standard_normal(n)), dev(torch, rng.standard_normal(n))
    vals = {v.dot(x, y) for _ in range(5)}
    assert len(vals) == 1
    ref = float(r32(host(x)) @ r32(host(y)))
    assert next(iter(vals)) == pytest.approx(ref, rel=1e-12)
