"""Shared helpers of the GPU tests: run the library through the C ABI on synthetic inputs."""
import numpy as np

import paper_2403_18840_amd as dmc

BETA, MU, LAM = 25.0, 1.0, 1.0


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def to_soa(x_np):
    """[N, D] float32 host -> [D, N] float32 device."""
    torch, dev = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x_np, dtype=np.float32).T)).to(dev)


def gpu_integrand(graph, x_np, ks, inst, jac=None):
    """Captured f (no Jacobian) [n_groups][n_roots][K][N] complex128, plus the accumulator."""
    torch, dev = torch_dev()
    N = x_np.shape[0]
    X = to_soa(x_np)
    J = torch.ones(N, dtype=torch.float32, device=dev) if jac is None else \
        torch.from_numpy(np.asarray(jac, dtype=np.float32)).to(dev)
    lams = []
    for p in inst:
        if p[2] not in lams:
            lams.append(p[2])
    G, K, R = len(lams), len(ks), graph.n_roots
    acc = dmc.Accumulator(G, K, R)
    f = torch.full((G * R * K * 2 * N,), float("nan"), dtype=torch.float32, device=dev)
    imp = torch.zeros(N, dtype=torch.float32, device=dev)
    dmc.eval_batch(graph, inst, ks, X, J, acc, f_out=f, imp_out=imp)
    dmc.accumulate(acc)
    torch.cuda.synchronize()
    fr = f.view(G, R, K, 2, N).cpu().numpy().astype(np.float64)
    return fr[:, :, :, 0, :] + 1j * fr[:, :, :, 1, :], acc, imp.cpu().numpy()


def parity_points(n, N, seed):
    """Per-sample parity inputs [N, D] float32.  Orders 1-3: the default draw.  Orders >= 4: half the rows
    from the default draw (with its edge cases), half with every loop momentum within 0.05 of the Fermi
    surface.  With momenta anywhere in the ball, the product of many propagators at beta = 25 puts most
    order-4..6 samples far below the 1e-30 floor of the per-sample rule; on the shell the integrand is
    1e-15..1e-10 at order 6, so the rule's relative part is what decides."""
    import synth
    if n <= 3:
        return synth.loop_points(n, N, seed=seed)
    h = N // 2
    return np.concatenate([synth.loop_points(n, h, seed=seed),
                           synth.loop_points(n, N - h, seed=seed + 7919, fermi_fraction=1.0, special=False)])
