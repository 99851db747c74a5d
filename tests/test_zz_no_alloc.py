"""The allocation-free evaluation entry point (dmc_eval_accumulate_noalloc, through the C ABI) against
dmc_eval_batch + dmc_accumulate on the same inputs: FP64 sums, counts, captured integrand and importance,
on two calls in a row (the second with fewer samples, so the static scratch holds the first call's
larger contents), for a single-part kernel and a kernel in parts with several lambda groups."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc

pytestmark = pytest.mark.gpu

BETA, MU = 25.0, 1.0


def _inputs(order, N, seed):
    import torch
    dev = torch.device("cuda:0")
    s = dmc.Sampler(dmc.SAMPLER_UNIFORM, order, n_bins=50, beta=BETA, qmax=6.0)
    X = torch.empty((dmc.dim(order), N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(seed, 0, X, J)
    return X, J


@pytest.mark.parametrize("order,mask,lams,K", [(3, 0, [1.0], 32), (5, dmc.D_K, [0.5, 1.0, 2.0], 9)])
def test_noalloc_matches_eval_batch(order, mask, lams, K):
    import torch
    dev = torch.device("cuda:0")
    g = dmc.Graph(order, deriv_mask=mask, deriv_k=1 if mask else 0)
    ks = np.linspace(0.0, 3.0, K).astype(np.float32)
    inst = [(BETA, MU, lam, dmc.coupling(rs)) for lam in lams for rs in (1.0, 3.0)]
    G, R = len(lams), g.n_roots
    with pytest.raises(dmc.DmcError) as e:   # the kernel is not loaded yet: the entry point compiles nothing
        dmc.eval_accumulate_noalloc(g, inst, ks, *_inputs(order, 256, 1), dmc.Accumulator(G, K, R))
    assert e.value.status == -5
    for call, N in enumerate([300_000 if order == 3 else 20_000, 70_001 if order == 3 else 3_001]):
        X, J = _inputs(order, N, 7 + call)
        acc_a, acc_b = dmc.Accumulator(G, K, R), dmc.Accumulator(G, K, R)
        fa = torch.zeros(G * R * K * 2 * N, dtype=torch.float32, device=dev)
        fb = torch.full_like(fa, float("nan"))
        ia = torch.zeros(N, dtype=torch.float32, device=dev)
        ib = torch.full_like(ia, float("nan"))
        dmc.eval_batch(g, inst, ks, X, J, acc_a, f_out=fa, imp_out=ia)
        dmc.accumulate(acc_a)
        dmc.eval_accumulate_noalloc(g, inst, ks, X, J, acc_b, f_out=fb, imp_out=ib)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb) and torch.equal(ia, ib)
        sa, na = acc_a.read()
        sb, nb = acc_b.read()
        assert na == nb == N
        assert np.allclose(sb, sa, rtol=1e-12, atol=1e-300)
        ma, ea, nsa, nfa = acc_a.estimate(len(inst))
        mb, eb, nsb, nfb = acc_b.estimate(len(inst))
        assert nsa == nsb == N and nfa == nfb
        assert np.allclose(mb, ma, rtol=1e-12, atol=1e-300) and np.allclose(eb, ea, rtol=1e-10, atol=1e-300)
        # a second call on the same accumulator keeps adding, like eval_batch + accumulate
        dmc.eval_accumulate_noalloc(g, inst, ks, X, J, acc_b)
        dmc.eval_batch(g, inst, ks, X, J, acc_a)
        dmc.accumulate(acc_a)
        assert acc_b.read()[1] == acc_a.read()[1] == 2 * N
        assert np.allclose(acc_b.read()[0], acc_a.read()[0], rtol=1e-12, atol=1e-300)
