"""Throughput of the diagrammatic Monte Carlo hot path on one MI355X.

Workload (the default): all connected 1PI self-energy diagrams of orders 1-3, bare Yukawa
lambda = 1, r_s in {1, 2} (one evaluated lambda; r_s enters as gamma^n), beta E_F = 25, 32
external |k| in [0, 3 k_F], VEGAS with 50 bins per dimension, 2^24 samples per iteration per
order, FP32 evaluation and FP64 accumulation.  One step = one VEGAS iteration over every order:
Philox sampling through the grid, graph evaluation, FP64 fold, estimate.  Warmup iterations
adapt the grid (histogram + refinement); timed iterations use the frozen grid.

Prints one JSON line (metric samples*diagrams/s = samples x diagrams x k x evaluated lambda per
second), with the roofline of the dominant kernel (the order-3 graph evaluation) measured with
HIP events on its stream, and the CPU oracle timed on a bounded sample of the same workload.

After the timed steps (outside them), `flow_vs_vegas` compares the learned proposal with VEGAS at
order 4 (D = 15): the error of Re Sigma(k_F, i omega_0) (scatter of 64 independent batch means of 2^22) and
wall time for the same number of samples from the adapted grid and from the trained 8-layer
affine-coupling flow (defensive mixture 0.85 flow + 0.10 grid + 0.05 uniform), the efficiency
(sigma_V^2 T_V) / (sigma_F^2 T_F) with and without adaptation and training time, and the flow
sampler's matrix-core roofline.  Then `mcmc_vs_vegas` compares, at order 2 by default, plain VEGAS
importance sampling with VEGAS-MCMC and NF-MCMC (independent proposals from the frozen grid or the
trained flow, target alpha q + (1 - alpha)|f|) over a sweep of alpha, at equal evaluation counts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X's published FP32 vector peak (dense)
PEAK_ALU_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz: the unpacked issue rate (packed FP32 is off)
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 matrix-core peak
# affine-coupling flow, 8 layers of 16 -> 128 -> 128 -> 32 (FMA = 2 FLOP); the products as executed


def affine_flow_flop(masks):
    """Algorithmic FLOP per sample of the affine flow (multiply-add = 2): per layer the network on the dA
    conditioning inputs plus the bias input, its 128 x 128 hidden product, and the 2 dB outputs (s and t of the
    transformed dimensions).  The kernel's MFMA tiles pad the input to 16 and the output to 32."""
    return sum(2 * ((int(m.sum()) + 1) * 128 + 128 * 128 + 128 * 2 * (len(m) - int(m.sum()))) for m in masks)


def flops(ops):
    """add, mul, fma, trans -> FLOP with FMA = 2."""
    return ops[0] + ops[1] + 2 * ops[2] + ops[3]


def traffic_for(graph, n_groups=1, n_samples=None, name="eval_o3_hbm_traffic.json"):
    """HBM bytes per launch from the committed counter runs (profiles/<name>), if the generated kernel is the one
    that was measured (same source) on as many samples, else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    src = graph.source(n_groups)
    if hashlib.sha1(src.encode()).hexdigest() != d.get("kernel_source_sha1"):
        return None
    if n_samples is not None and d.get("samples_per_launch") not in (None, n_samples):
        return None
    return d["hbm_bytes_per_launch"]


def _oracle_times(orders, K, per, beta, mu, lam, gamma, seed0=1000):
    """Per order: (samples done, seconds spent) of the oracle (numpy FP64, diagram by diagram) on about
    `per` seconds of work, batches doubling from 256 samples."""
    import numpy as np

    import synth
    from oracle import integrand as ig

    ks = synth.k_grid(K)
    out = []
    for n in orders:
        N, spent, done = 256, 0.0, 0
        while spent < per:
            x = synth.loop_points(n, N, seed=seed0 + n + done).astype(np.float64)
            t0 = time.perf_counter()
            for k in ks:
                ig.integrand(x, n, float(k), beta, mu, lam, gamma)
            spent += time.perf_counter() - t0
            done += N
            N = min(N * 2, 1 << 15)
        out.append((done, spent))
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(orders, K, seconds, beta, mu, lam, gamma, workers=0):
    """The oracle (numpy FP64, diagram by diagram) on a bounded sample of each order, on one thread.  The
    rate is combined with the workload's mix (equal samples per order): value = sum_n N_diag(n) / sum_n t_n,
    t_n being the oracle's seconds per (sample, k) at order n.  With workers > 1 the same loop also runs in
    that many child processes at once (disjoint samples; they touch no GPU), t_n = the slowest worker's
    seconds / all workers' (samples x K): the rate on the host's cores."""
    import subprocess

    from oracle import diagrams as dg

    per = seconds / len(orders)
    nds = [len(dg.sigma_diagrams(n)) for n in orders]
    times = _oracle_times(orders, K, per, beta, mu, lam, gamma)
    t_per = sum(sp / (dn * K) for dn, sp in times)
    desc = [f"order {n}: {dn} samples x {K} k in {sp:.1f} s" for n, (dn, sp) in zip(orders, times)]
    out = {"value": sum(nds) / t_per, "unit": "samples·diagrams/s", "cores": 1, "kind": "oracle",
           "sample": "; ".join(desc) + " (numpy FP64, one thread; rate combined with equal samples per order)",
           "cpu_model": _cpu_model()}
    if workers > 1:
        code = ("import json, sys; sys.path.insert(0, %r); import bench; "
                "print(json.dumps(bench._oracle_times(%r, %d, %r, %r, %r, %r, %r, seed0=%%d)))"
                % (os.path.dirname(os.path.abspath(__file__)), list(orders), K, per / 2, beta, mu, lam, gamma))
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
        t0 = time.perf_counter()
        procs = [subprocess.Popen([sys.executable, "-c", code % (100000 * (w + 1))], stdout=subprocess.PIPE,
                                  env=env, text=True) for w in range(workers)]
        res = []
        for p in procs:
            o, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError("oracle worker failed")
            res.append(json.loads(o.strip().splitlines()[-1]))
        wall = time.perf_counter() - t0
        t_all = 0.0
        for i in range(len(orders)):
            done = sum(r[i][0] for r in res)
            t_all += max(r[i][1] for r in res) / (done * K)
        out["all_cores"] = {"value": sum(nds) / t_all, "cores": workers, "wall_seconds": wall,
                            "sample": f"{workers} processes x {per / 2:.1f} s per order, disjoint samples"}
    return out


def measured_peaks():
    """The roofline denominators measured on this device (dmc_probe): unpacked FP32 FMA (TFLOP/s, FMA = 2),
    the hardware 2^x and reciprocal (operations per compute unit and clock at the 2.4 GHz peak clock), and a
    1 GiB device copy (TB/s, bytes read plus written).  Best of three launches each."""
    import paper_2403_18840_amd as dmc

    def best(kind, work):
        runs = [dmc.probe(kind, work) for _ in range(3)]
        return max(o / (m * 1e-3) for m, o in runs)

    per_clk = 256 * 2.4e9
    return {"fp32_fma_tflops": 2 * best(0, 4096) / 1e12, "exp2_per_cu_clock": best(1, 1024) / per_clk,
            "rcp_per_cu_clock": best(2, 1024) / per_clk, "fma_per_cu_clock": best(0, 4096) / per_clk,
            "hbm_copy_tbs": best(3, 1 << 30) / 1e12,
            "assumed": {"fp32_vector_tflops": PEAK_FP32_TFLOPS, "fp32_unpacked_tflops": PEAK_ALU_TFLOPS, "hbm_tbs": 8.0,
                        "clock_ghz": 2.4, "cus": 256}}


def _make_flow(D, kind):
    """The learned proposal: "affine" (8 affine couplings, 128-wide MLPs, BF16 matrix cores; He-normal hidden
    weights, zero output layer) or "spline" (the paper's flow: 6 rational-quadratic spline couplings with
    8 bins and a residual conditioner of two 32-unit layers; the library's identity start)."""
    import paper_2403_18840_amd as dmc
    import synth
    if kind == "spline":
        return dmc.Flow(D, synth.flow_masks(D, 6, 5), kind="spline")
    masks = synth.flow_masks(D, 8, 5)
    f = dmc.Flow(D, masks)
    f.set_params(synth.flow_params(masks, 6, last_scale=0.0))
    return f


def flow_vs_vegas(order, K, N, batches, beta, mu, lam, gamma, seed=0x2403188400000004, train="is", kind="affine",
                  graph=None, inst=None, ks=None, epochs=4, steps=64):
    """Learned proposal at one order: Re Sigma(k_F, i omega_0) from `batches` independent batches of N
    samples drawn from the adapted VEGAS grid alone and from the trained flow's defensive mixture
    (0.85 flow + 0.10 grid + 0.05 uniform), each with its wall time (GPU-synchronised).  sigma is the
    scatter of the batch means / sqrt(batches): at this order the weights are heavy-tailed and the
    in-run sample sigma understates the error (both are reported), and a few batches can dominate
    the scatter, so the robust spread (1.4826 x the median absolute deviation of the batch means)
    is reported beside it.  Efficiency = (sigma_V^2 T_V) / (sigma_F^2 T_F), without and with
    adaptation + training time.  train = "is": the flow learns from importance-weighted draws of the
    grid and then of its own mixture (train_flow); "mcmc": from Markov-chain samples of |f| with
    proposals from its mixture (train_flow_mcmc), with the same number of Adam steps."""
    import numpy as np
    import torch

    import paper_2403_18840_amd as dmc
    import synth

    dev = torch.device("cuda:0")
    ks = np.linspace(0.0, 3.0, K).astype(np.float32) if ks is None else np.asarray(ks, dtype=np.float32)
    jf = int(np.argmin(np.abs(ks - 1.0)))
    inst = [(beta, mu, lam, gamma)] if inst is None else inst
    # the figure of merit: Re Sigma(k_F) of the instance with this lambda and gamma
    i_fom = [i for i, p in enumerate(inst) if p[2] == lam and p[3] == gamma][0]
    groups = len(set(p[2] for p in inst))
    D = dmc.dim(order)
    g = dmc.Graph(order) if graph is None else graph
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, order, n_bins=50, beta=beta, qmax=6.0)
    a_f, a_u = 0.85, 0.05

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    _, t_adapt = timed(lambda: dmc.adapt_grid(g, inst, ks, s, 1 << 22, 6, seed=seed))
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)

    imp = torch.empty(N, dtype=torch.float32, device=dev)

    def run(draw):
        means, sig, nonfin, ess, wmax = [], [], 0, [], []
        for b in range(batches):
            acc = dmc.Accumulator(groups, len(ks), g.n_roots)
            draw(b)
            dmc.eval_batch(g, inst, ks, X, J, acc, imp_out=imp)
            dmc.accumulate(acc)
            m, e, _, nf = acc.estimate(len(inst))
            means.append(m[i_fom, 0, jf].real)
            sig.append(e[i_fom, 0, jf].real)
            nonfin += nf
            # weight diagnostics of the batch from its importances (sum over k, Re/Im of |f| J): the effective
            # sample size fraction (sum w)^2 / (N sum w^2) and the largest weight over the mean
            w = imp.double()
            s1, s2 = float(w.sum()), float((w * w).sum())
            ess.append(s1 * s1 / (N * s2) if s2 > 0 else 0.0)
            wmax.append(float(w.max()) * N / s1 if s1 > 0 else 0.0)
        means = np.array(means)
        mad = 1.4826 * float(np.median(np.abs(means - np.median(means))))
        return {"re": float(means.mean()), "sigma": float(means.std(ddof=1) / math.sqrt(batches)),
                "sigma_mad": mad / math.sqrt(batches),
                "sigma_in_run": float(math.sqrt(np.mean(np.square(sig)) / batches)), "nonfinite": int(nonfin),
                "ess_fraction_median": float(np.median(ess)), "max_weight_over_mean_median": float(np.median(wmax)),
                "max_weight_over_mean_max": float(np.max(wmax))}

    vg, t_v = timed(lambda: run(lambda b: s.sample(seed + 1, b * N, X, J)))
    f = _make_flow(D, kind)
    mb = 1 << 17
    if train == "mcmc":
        losses, t_train = timed(lambda: dmc.train_flow_mcmc(g, inst, ks, s, f, rounds=epochs, n_chains=mb, thermal=200,
                                                             collect=8, stride=10, steps=steps, lr=1e-3,
                                                             flow_alpha=a_f, flow_uniform=a_u, seed=seed + 2))
    else:
        losses, t_train = timed(lambda: dmc.train_flow(g, inst, ks, s, f, epochs=epochs, steps=steps, minibatch=mb,
                                                        lr=1e-3, alpha=a_f, uniform=a_u, seed=seed + 2))
    fl, t_f = timed(lambda: run(lambda b: f.sample(s, seed + 3, b * N, X, J, alpha=a_f, uniform=a_u)))
    # the sampler kernel alone (all N samples through the flow), HIP events on its stream
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    for i, (a, b) in enumerate(evs):
        a.record(stream)
        f.sample(s, seed + 4, i * N, X, J, alpha=1.0)
        b.record(stream)
    torch.cuda.synchronize()
    k_ms = sum(a.elapsed_time(b) for a, b in evs) / len(evs)
    if kind == "spline":
        # conditioner multiply-adds per sample (2 FLOP each): 32 dA + 32 x 32 + 23 dB x 32 per layer
        per = sum(2 * (32 * int(m.sum()) + 32 * 32 + 23 * (D - int(m.sum())) * 32) for m in f.masks)
        flop, peak, bound, kname = N * per, PEAK_FP32_TFLOPS, "alu", f"dmc_nsf_sample_kernel (D = {D})"
    else:
        flop, peak, bound, kname = N * affine_flow_flop(f.masks), PEAK_BF16_TFLOPS, "mfma", f"dmc_flow_sample_kernel<{D}>"
    ev, ef = vg["sigma"], fl["sigma"]
    vg["seconds"] = t_v
    fl.update({"seconds": t_f, "kind": kind, "layers": f.n_layers,
               "mixture": {"flow": a_f, "grid": 1 - a_f - a_u, "uniform": a_u},
               "training": {"kind": train, "adam_steps": epochs * steps, "minibatch": mb, "seconds": t_train,
                            "loss": [float(x) for x in losses]}})
    return {
        "order": order, "k": float(ks[jf]), "samples_per_batch": N, "batches": batches,
        "vegas": vg, "flow": fl, "adapt_seconds": t_adapt,
        "roofline": {"bound": bound, "kernel": kname, "achieved": flop / (k_ms * 1e-3) / 1e12,
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": flop / (k_ms * 1e-3) / 1e12 / peak, "kernel_ms": k_ms,
                     "flop_per_launch": flop},
        # ratios of spreads are undefined with a single batch (zero spread): null
        "z": _ratio(vg["re"] - fl["re"], math.hypot(ev, ef)),
        "variance_ratio": _ratio(ev ** 2, ef ** 2),
        "variance_ratio_mad": _ratio(vg["sigma_mad"] ** 2, fl["sigma_mad"] ** 2),
        "efficiency_steady": _ratio(ev ** 2 * t_v, ef ** 2 * t_f),
        "efficiency_total": _ratio(ev ** 2 * (t_adapt + t_v), ef ** 2 * (t_adapt + t_train + t_f)),
    }


def routing_compare(orders, n_samples=1 << 22, reps=5, ks_list=(1, 32)):
    """Path routing against building-block variables (dmc_graph_spec.routing): eval_batch + accumulate of one
    lambda group on n_samples uniform samples, at one external momentum (k_F) and at 32 in [0, 3 k_F]; the mean of
    `reps` launches by HIP events, with each graph's executed op counts per sample and per (sample, k)."""
    import numpy as np
    import torch

    import paper_2403_18840_amd as dmc

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    inst = [(25.0, 1.0, 1.0, dmc.coupling(1.0))]
    rows = []
    for n in orders:
        s = dmc.Sampler(dmc.SAMPLER_UNIFORM, n)
        X = torch.empty((dmc.dim(n), n_samples), dtype=torch.float32, device=dev)
        J = torch.empty(n_samples, dtype=torch.float32, device=dev)
        s.sample(1, 0, X, J)
        for routing, name in ((dmc.ROUTING_PATH, "path"), (dmc.ROUTING_BLOCKS, "blocks")):
            g = dmc.Graph(n, routing=routing)
            info = g.info()
            for K in ks_list:
                ks = np.array([1.0], dtype=np.float32) if K == 1 else np.linspace(0.0, 3.0, K).astype(np.float32)
                acc = dmc.Accumulator(1, K, 1)
                dmc.eval_batch(g, inst, ks, X, J, acc, stream=stream)
                dmc.accumulate(acc, stream=stream)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(reps):
                    dmc.eval_batch(g, inst, ks, X, J, acc, stream=stream)
                    dmc.accumulate(acc, stream=stream)
                b.record(stream)
                torch.cuda.synchronize()
                rows.append({"order": n, "routing": name, "n_k": K, "samples": n_samples,
                             "ms": a.elapsed_time(b) / reps, "parts": info.n_parts,
                             "ops_sample_exec": int(sum(info.ops_sample_exec)), "ops_k_exec": int(sum(info.ops_k_exec))})
                print(f"[routing] {name} order {n} K {K}: {rows[-1]['ms']:.3f} ms", file=sys.stderr, flush=True)
    return rows


def _ratio(a, b):
    return float(a / b) if b > 0 and math.isfinite(b) else None


def mcmc_vs_vegas(order, beta, mu, lam, gamma, n_chains=1 << 16, steps=1024, thermal=2000, n_batches=64,
                  alphas=(0.05, 0.2, 0.5, 0.8), seed=0x2403188400000005, flow=True, ref_factor=16, flow_kind="affine",
                  walk_every=2, walk_sigma=0.05):
    """Markov-chain estimators against plain VEGAS importance sampling at one order (the comparison
    of Sec. IV): Re Sigma(k_F, i omega_0) alone (K = 1, so p = |Re f| + |Im f| at k_F).  VEGAS IS:
    ref_factor x n_batches batches of n_chains * steps / n_batches samples from the adapted grid; the
    scatter of the batch means gives sigma at the chains' evaluation count (sigma_b / sqrt(n_batches))
    and the reference for the z of each chain estimate (sigma_b / sqrt(ref_factor n_batches)); the
    weights are heavy-tailed from order 3 on, so the robust spread (1.4826 x the median absolute
    deviation of the batch means) is reported beside it.  VEGAS-MCMC (the frozen grid as independent
    proposal) and, with `flow`, NF-MCMC (the trained flow's defensive mixture as proposal), for each mixing parameter alpha:
    n_chains chains, `thermal` steps discarded, `steps` measured, sigma from n_batches independent
    chain batches.  Equal evaluation counts: the efficiency relative to VEGAS is
    sigma_VEGAS^2 / sigma^2 per evaluation and sigma_VEGAS^2 T_VEGAS / (sigma^2 T) per wall second
    (the thermalisation steps count in T).  With a spline flow and walk_every > 0, NF-MCMC runs a second
    time with every walk_every-th step a random-walk move of step walk_sigma in the flow's base space."""
    import numpy as np
    import torch

    import paper_2403_18840_amd as dmc
    import synth

    dev = torch.device("cuda:0")
    ks = np.array([1.0], dtype=np.float32)
    inst = [(beta, mu, lam, gamma)]
    D = dmc.dim(order)
    g = dmc.Graph(order)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, order, n_bins=50, beta=beta, qmax=6.0)
    n_eval = n_chains * steps

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def log(msg):
        print(f"[mcmc order {order}] {msg}", file=sys.stderr, flush=True)

    _, t_adapt = timed(lambda: dmc.adapt_grid(g, inst, ks, s, 1 << 22, 6, seed=seed))
    nb = n_eval // n_batches
    X = torch.empty((D, nb), dtype=torch.float32, device=dev)
    J = torch.empty(nb, dtype=torch.float32, device=dev)

    def vegas_is():
        means = []
        for b in range(n_batches * ref_factor):
            acc = dmc.Accumulator(1, 1, 1)
            s.sample(seed + 1, b * nb, X, J)
            dmc.eval_batch(g, inst, ks, X, J, acc)
            dmc.accumulate(acc)
            m, _, _, _ = acc.estimate(1)
            means.append(m[0, 0, 0].real)
        means = np.array(means)
        sb = float(means.std(ddof=1))
        mad = 1.4826 * float(np.median(np.abs(means - np.median(means))))
        return (float(means.mean()), sb / math.sqrt(n_batches), sb / math.sqrt(n_batches * ref_factor),
                mad / math.sqrt(n_batches))

    (v_re, v_sig, v_ref, v_mad), t_ref = timed(vegas_is)
    t_v = t_ref / ref_factor
    log(f"VEGAS IS {v_re:.6g} +- {v_ref:.3g} ({ref_factor} x {n_eval} evaluations, {t_ref:.2f} s); "
        f"sigma at {n_eval}: {v_sig:.3g} (robust {v_mad:.3g})")
    out = {"order": order, "k": 1.0, "evaluations": n_eval, "n_chains": n_chains, "steps": steps,
           "thermal": thermal, "n_batches": n_batches, "adapt_seconds": t_adapt,
           "vegas": {"re": v_re, "sigma_ref": v_ref, "ref_factor": ref_factor, "sigma": v_sig, "sigma_mad": v_mad,
                     "seconds": t_v}}

    def chains(label, fl, walk=0):
        rows = []
        for a in alphas:
            r, t = timed(lambda: dmc.mcmc_integrate(g, inst, ks, s, n_chains, steps, thermal=thermal, alpha=a,
                                                    seed=seed + 7, n_batches=n_batches, flow=fl, walk_every=walk,
                                                    walk_sigma=walk_sigma))
            re, sig = float(r.mean[0, 0, 0].real), float(r.err[0, 0, 0].real)
            zh = float(r.halves[2][0, 0, 0].real)
            rows.append({"alpha": a, "re": re, "sigma": sig, "acceptance": r.acceptance, "seconds": t,
                         "efficiency_per_eval": (v_sig / sig) ** 2, "efficiency_per_eval_mad": (v_mad / sig) ** 2,
                         "efficiency_per_second": (v_sig ** 2 * t_v) / (sig ** 2 * t),
                         "z_vs_vegas": (re - v_re) / math.hypot(sig, v_ref), "z_halves": zh,
                         "proposal_is": {"re": float(r.is_mean[0, 0, 0].real), "sigma": float(r.is_err[0, 0, 0].real)}})
            log(f"{label} alpha {a}: {re:.6g} +- {sig:.3g} (z vs VEGAS {rows[-1]['z_vs_vegas']:+.2f}, halves {zh:+.2f}), "
                f"acceptance {r.acceptance:.3f}, efficiency/eval {(v_sig / sig) ** 2:.2f} "
                f"(robust {(v_mad / sig) ** 2:.2f}) ({t:.2f} s)")
        # best alpha among the runs that agree with VEGAS and show no trend between their halves
        ok = [r for r in rows if abs(r["z_vs_vegas"]) < 3 and abs(r["z_halves"]) < 3]
        best = max(ok, key=lambda r: r["efficiency_per_eval"]) if ok else None
        return {"alphas": rows, "best_alpha": best and best["alpha"],
                "best_efficiency_per_eval": best and best["efficiency_per_eval"],
                "best_efficiency_per_second": best and best["efficiency_per_second"]}

    out["vegas_mcmc"] = chains("VEGAS-MCMC", None)
    if flow:
        f = _make_flow(D, flow_kind)
        epochs, tsteps, mb = 4, 64, 1 << 17
        losses, t_train = timed(lambda: dmc.train_flow(g, inst, ks, s, f, epochs=epochs, steps=tsteps, minibatch=mb,
                                                        lr=1e-3, seed=seed + 2))
        log(f"flow trained ({t_train:.1f} s), losses {[round(float(x), 3) for x in losses]}")
        out["nf_mcmc"] = chains("NF-MCMC", f)
        out["nf_mcmc"]["training"] = {"samples": epochs * tsteps * mb, "seconds": t_train, "kind": flow_kind,
                                      "loss": [float(x) for x in losses], "mixture": {"flow": 0.85, "uniform": 0.05}}
        if flow_kind == "spline" and walk_every > 0:
            out["nf_mcmc_walk"] = chains("NF-MCMC + walk", f, walk=walk_every)
            out["nf_mcmc_walk"].update({"walk_every": walk_every, "walk_sigma": walk_sigma})
    return out


def effective_mass_leg(N, rs, lam_R, beta, log2_samples, batches):
    """The renormalised m*/m series through total order N (Sec. VI.A): Taylor-mode graphs at each
    order n <= N (every d^m/dmu^m d^l/dlambda^l with m + l <= N - n, and the k derivatives), VEGAS
    at k_F, the counterterm recursion and the xi series in the library; jackknife errors over
    independent batches.  Reports each order's partial sum with its error and the wall time."""
    import torch

    import paper_2403_18840_amd as dmc

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mp, me, dm, de = dmc.effective_mass_estimate(N, rs, lam_R, beta=beta, n_samples=1 << log2_samples,
                                                 batches=batches)
    torch.cuda.synchronize()
    return {"order": N, "rs": rs, "lambda_R": lam_R, "beta": beta, "samples_per_batch": 1 << log2_samples,
            "batches": batches, "mass_partial": [float(v) for v in mp], "mass_partial_err": [float(v) for v in me],
            "delta_mu": [float(v) for v in dm], "delta_mu_err": [float(v) for v in de],
            "seconds": time.perf_counter() - t0}


def cpu_baseline_c5(order, ks, lams, beta, mu, gamma, seconds=15.0):
    """The oracle's C integrand (oracle/evaluate.c: FP64, diagram by diagram, OpenMP over samples on the host's
    threads) on a bounded sample of the order-n workload: samples drawn like the tests' inputs, every lambda
    group, the momenta ks; batches double until about `seconds` of work.  Rate in samples x diagrams x k x
    lambda per second."""
    import numpy as np

    import synth
    from oracle import cevaluate as ce
    from golden_diagrams import oracle_diagrams

    dgs = oracle_diagrams(order)
    tab = ce.table(dgs, order)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    N, done, spent = 16, 0, 0.0
    while spent < seconds:
        x = synth.loop_points(order, N, seed=4000 + done).astype(np.float64)
        t0 = time.perf_counter()
        for lam in lams:
            for k in ks:
                ce.evaluate(x, order, float(k), beta, mu, lam, gamma, dgs, tab=tab)
        spent += time.perf_counter() - t0
        done += N
        N = min(2 * N, 4096)
    units = done * len(dgs) * len(ks) * len(lams)
    return {"value": units / spent, "unit": "samples·diagrams/s", "cores": threads, "kind": "oracle",
            "sample": f"order {order}: {done} samples x {len(ks)} k x {len(lams)} lambda in {spent:.1f} s "
                      f"(C FP64 diagram-by-diagram integrand, OpenMP, {threads} threads)",
            "cpu_model": _cpu_model()}


def run_c5(args):
    """The order-6 effective-mass workload: all 31130 order-6 diagrams, d Sigma / dk at k_F (the effective mass'
    a coefficient), lambda in {0.5, 1, 2} with r_s 1..5 as gamma^n rescalings (15 instances, 3 evaluated), one
    launch for all of them; importance sampling from the trained affine flow's defensive mixture; 2^26 samples
    per iteration.  One step = one iteration: flow sampling, evaluation, FP64 fold, estimate."""
    import numpy as np
    import torch

    import paper_2403_18840_amd as dmc
    import synth

    dev = torch.device("cuda:0")
    order, beta, mu = 6, 25.0, 1.0
    lams, rs_list = [0.5, 1.0, 2.0], [1.0, 2.0, 3.0, 4.0, 5.0]
    inst = [(beta, mu, lam, dmc.coupling(rs)) for lam in lams for rs in rs_list]
    # k_F first (it carries the derivative root), then 32 momenta in [0, 3 k_F]
    ks = np.concatenate([[1.0], np.linspace(0.0, 3.0, 32)]).astype(np.float32)
    K = len(ks)
    N = 1 << args.log2_samples
    D = dmc.dim(order)
    t_setup = time.perf_counter()
    g = dmc.Graph(order, deriv_mask=dmc.D_K, deriv_k=1)
    inf = g.info()
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, order, n_bins=50, beta=beta, qmax=6.0)
    log = lambda m: print(f"[c5] {m}", file=sys.stderr, flush=True)
    seed0 = 0x2403188400000005
    # setup (untimed): adapt the grid, then train the flow on it (the first evaluation compiles the kernel)
    nxt = dmc.adapt_grid(g, inst, ks, s, 1 << 21, 4, seed=seed0)
    log(f"grid adapted ({time.perf_counter() - t_setup:.1f} s incl. compilation)")
    masks = synth.flow_masks(D, 8, 5)
    flow = dmc.Flow(D, masks)
    flow.set_params(synth.flow_params(masks, 6, last_scale=0.0))
    a_f, a_u = 0.85, 0.05
    losses = dmc.train_flow(g, inst, ks, s, flow, epochs=args.c5_train_epochs, steps=32, minibatch=1 << 17, lr=1e-3,
                            alpha=a_f, uniform=a_u, seed=seed0 + 1)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log(f"flow trained, setup {t_setup:.1f} s, losses {[round(float(x), 3) for x in losses]}")
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    acc = dmc.Accumulator(len(lams), K, g.n_roots)
    stream = torch.cuda.current_stream()
    state = {}

    def step(it, ev=None):
        acc.reset()
        flow.sample(s, seed0 + 2, it * N, X, J, alpha=a_f, uniform=a_u)
        if ev is not None:
            ev[0].record(stream)
        dmc.eval_batch(g, inst, ks, X, J, acc)
        if ev is not None:
            ev[1].record(stream)
        dmc.accumulate(acc)
        state["last"] = acc.estimate(len(inst))
        if ev is not None:
            state.setdefault("iters", []).append(state["last"])

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, ev=evs[i])
        if (i + 1) % 10 == 0:
            log(f"{i + 1} of {args.steps} timed iterations")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    units = N * inf.n_diagrams * K * len(lams)
    # algorithmic FLOP per launch: per lambda group, the k-independent graph once per sample, the value's
    # k-dependent part at every momentum and the derivative-only part at k_F (FMA = 2)
    per_group = flops(list(inf.ops_sample)) + K * (flops(list(inf.ops_k)) - flops(list(inf.ops_k_deriv))) \
        + 1 * flops(list(inf.ops_k_deriv))
    fl_launch = N * len(lams) * per_group
    achieved = fl_launch / (kern_ms * 1e-3) / 1e12
    i1 = inst.index((beta, mu, 1.0, dmc.coupling(1.0)))
    w0 = math.pi / beta
    # the timed iterations combined with equal weights (dmc_combine_iterations): Re, Im of Sigma and of d Sigma/dk
    # at k_F for lambda = 1, r_s = 1
    its = state["iters"]
    pick = lambda a: [a[i1, 0, 0].real, a[i1, 0, 0].imag, a[i1, 1, 0].real, a[i1, 1, 0].imag]
    cm, ce, chi = dmc.combine_iterations([pick(it[0]) for it in its], [pick(it[1]) for it in its])
    nf = int(sum(it[3] for it in its))
    out = {
        "metric": "samples·diagrams/s",
        "value": units / dt,
        "unit": "samples·diagrams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"UEG self-energy order 6 (all {inf.n_diagrams} 1PI diagrams, D = 23) with d Sigma/dk at k_F, "
                        f"Yukawa lambda 0.5/1/2 x r_s 1..5 (15 instances, 3 evaluated) in one launch, beta E_F = 25, "
                        f"{K} |k| (k_F and 32 in [0, 3 k_F]), affine-flow proposal (8 layers, 0.85 flow + 0.10 VEGAS "
                        f"grid + 0.05 uniform), 2^{args.log2_samples} samples/iteration",
            "order": order, "n_k": K, "samples_per_iteration": N, "lambda_evaluated": lams, "rs": rs_list,
            "derivative": "d/dk at k_F", "kernel_parts": inf.n_parts, "setup_seconds": t_setup,
        },
        "roofline": {
            "bound": "alu", "kernel": f"dmc_eval_o6_g3_r2 ({inf.n_parts} parts)", "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic_for(g, len(lams), N, "eval_o6_c5_hbm_traffic.json"),
            "kernel_ms": kern_ms, "flop_per_launch": fl_launch,
            "flop_per_sample_per_group": per_group,
            "frac_of_unpacked_issue_rate": achieved / PEAK_ALU_TFLOPS,
        },
        "estimate": {"lambda": 1.0, "rs": 1.0, "k": 1.0, "order": order, "iterations": len(its),
                     "re": float(cm[0]), "re_err": float(ce[0]), "im": float(cm[1]), "im_err": float(ce[1]),
                     "dre_dk": float(cm[2]), "dre_dk_err": float(ce[2]),
                     # the order-6 coefficients of the effective mass: a = (m/k_F) dRe/dk (m/k_F = 1/2), b = Im/w0
                     "a": 0.5 * float(cm[2]), "a_err": 0.5 * float(ce[2]), "b": float(cm[1]) / w0,
                     "b_err": float(ce[1]) / w0,
                     # chi^2/dof of the iterations about their combination (Re, Im, dRe/dk); nan with one iteration
                     "chi2_dof": [float(c) if math.isfinite(c) else None for c in chi[:3]],
                     "nonfinite": int(nf)},
    }
    if not args.no_peaks:
        out["peaks"] = measured_peaks()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_c5(order, [float(ks[0]), float(ks[1])], lams, beta, mu, dmc.coupling(1.0),
                                              seconds=args.cpu_seconds)
    if args.flow_order:
        log("flow vs VEGAS at order 6")
        out["flow_vs_vegas"] = flow_vs_vegas(order, K, 1 << args.flow_log2_samples, args.flow_batches, beta, mu,
                                             1.0, dmc.coupling(1.0), train=args.flow_train, kind=args.flow_kind,
                                             graph=g, inst=inst, ks=ks, epochs=args.c5_train_epochs, steps=32)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["c5", "c2"], default="c5",
                    help="c5: order 6 with d/dk at k_F, 3 lambda x 5 r_s, flow proposal, 2^26 samples (the default "
                         "line); c2: orders 1-3, r_s 1,2, VEGAS, 2^24 samples per order")
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (c5: 3, c2: 10)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed iterations first (c5: 1, c2: 5)")
    ap.add_argument("--orders", default="1,2,3")
    ap.add_argument("--log2-samples", type=int, default=None, help="samples per iteration (c5: 26, c2: 24)")
    ap.add_argument("--c5-train-epochs", type=int, default=3)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the throughput probes of the roofline denominators")
    ap.add_argument("--cpu-workers", type=int,
                    default=min(16, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))),
                    help="processes of the all-cores oracle timing (the host's CPU share; 1 or less skips it)")
    ap.add_argument("--flow-order", type=int, default=None,
                    help="order of the learned-proposal comparison (0 skips it; c5: 6, on its own graph; c2: 4)")
    ap.add_argument("--flow-batches", type=int, default=None)
    ap.add_argument("--flow-log2-samples", type=int, default=22)
    ap.add_argument("--flow-kind", choices=["affine", "spline"], default="affine",
                    help="learned proposal of the flow and NF-MCMC legs")
    ap.add_argument("--flow-train", choices=["is", "mcmc"], default="is",
                    help="training data of the flow: importance-weighted draws or Markov-chain samples of |f|")
    ap.add_argument("--mcmc-orders", default=None,
                    help="orders of the Markov-chain vs VEGAS comparison, comma-separated (empty skips it; "
                         "c5: empty, c2: 2)")
    ap.add_argument("--mcmc-log2-chains", type=int, default=16)
    ap.add_argument("--mcmc-steps", type=int, default=1024)
    ap.add_argument("--mcmc-thermal", type=int, default=2000)
    ap.add_argument("--mcmc-no-flow", action="store_true")
    ap.add_argument("--mcmc-walk-every", type=int, default=2,
                    help="with --flow-kind spline, also run NF-MCMC with every m-th step a base-space walk (0: off)")
    ap.add_argument("--mcmc-walk-sigma", type=float, default=0.05)
    ap.add_argument("--mass-order", type=int, default=0,
                    help="total order of the renormalised effective-mass series (0 skips it)")
    ap.add_argument("--mass-rs", type=float, default=1.0)
    ap.add_argument("--mass-lambda", type=float, default=1.0)
    ap.add_argument("--mass-log2-samples", type=int, default=22)
    ap.add_argument("--mass-batches", type=int, default=16)
    ap.add_argument("--routing-orders", default="",
                    help="orders at which to time path routing against building-block variables (empty skips it)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    c5 = args.workload == "c5"
    for name, v5, v2 in [("steps", 3, 10), ("warmup", 1, 5), ("log2_samples", 26, 24), ("flow_order", 6, 4),
                         ("flow_batches", 32, 64), ("mcmc_orders", "", "2")]:
        if getattr(args, name) is None:
            setattr(args, name, v5 if c5 else v2)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    if c5:
        import torch
        torch.cuda.set_device(torch.device("cuda:0"))
        if args.copy_mib:
            src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda:0")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        out = run_c5(args)
        if args.mcmc_orders:
            import paper_2403_18840_amd as dmc
            out["mcmc_vs_vegas"] = [mcmc_vs_vegas(int(n), 25.0, 1.0, 1.0, dmc.coupling(1.0),
                                                  n_chains=1 << args.mcmc_log2_chains, steps=args.mcmc_steps,
                                                  thermal=args.mcmc_thermal, flow=not args.mcmc_no_flow,
                                                  flow_kind=args.flow_kind, walk_every=args.mcmc_walk_every,
                                                  walk_sigma=args.mcmc_walk_sigma)
                                    for n in args.mcmc_orders.split(",")]
        if args.mass_order:
            out["effective_mass"] = effective_mass_leg(args.mass_order, args.mass_rs, args.mass_lambda, 25.0,
                                                       args.mass_log2_samples, args.mass_batches)
        if args.routing_orders:
            out["routing_compare"] = routing_compare([int(n) for n in args.routing_orders.split(",")])
        print(json.dumps(out), flush=True)
        return

    import numpy as np
    import torch

    import paper_2403_18840_amd as dmc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    orders = [int(t) for t in args.orders.split(",")]
    N = 1 << args.log2_samples
    K = args.k
    beta, mu, lam = 25.0, 1.0, 1.0
    rs_list = [1.0, 2.0]
    inst = [(beta, mu, lam, dmc.coupling(rs)) for rs in rs_list]
    ks = np.linspace(0.0, 3.0, K).astype(np.float32)
    Dmax = dmc.dim(max(orders))
    X = torch.empty((Dmax, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    imp = torch.empty(N, dtype=torch.float32, device=dev)
    runs = []
    for n in orders:
        g = dmc.Graph(n)
        s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50, beta=beta, qmax=6.0)
        acc = dmc.Accumulator(1, K, 1)
        runs.append(dict(n=n, g=g, s=s, acc=acc, info=g.info()))
    seed0 = 0x2403188400000001
    stream = torch.cuda.current_stream()

    def iteration(it, adapt, ev=None):
        # every order's sampling, evaluation and reduction is queued before the first estimate waits on the
        # stream (one synchronisation per step; the orders share X and J in stream order); an adapting
        # iteration refines each grid from its own histogram before the next order reuses imp
        for r in runs:
            n = r["n"]
            Xn = X.narrow(0, 0, dmc.dim(n))
            r["acc"].reset()
            r["s"].sample(seed0 + n, it * N, Xn, J)
            if ev is not None and n == orders[-1]:
                ev[0].record(stream)
            dmc.eval_batch(r["g"], inst, ks, Xn, J, r["acc"], imp_out=imp if adapt else None)
            if ev is not None and n == orders[-1]:
                ev[1].record(stream)
            dmc.accumulate(r["acc"], r["s"] if adapt else None, imp if adapt else None)
            if adapt:
                r["last"] = r["acc"].estimate(len(inst))[:2]
                r["s"].refine(0.5)
        if not adapt:
            for r in runs:
                r["last"] = r["acc"].estimate(len(inst))[:2]

    for w in range(args.warmup):
        iteration(w, adapt=True)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        iteration(args.warmup + i, adapt=False, ev=evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    units = sum(N * r["info"].n_diagrams * K * 1 for r in runs)
    dom = runs[-1]
    inf = dom["info"]
    fl_launch = N * (flops(list(inf.ops_sample)) + K * flops(list(inf.ops_k)))
    achieved = fl_launch / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "samples·diagrams/s",
        "value": units / dt,
        "unit": "samples·diagrams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"UEG self-energy orders {orders[0]}-{orders[-1]}, all 1PI diagrams "
                        f"({'+'.join(str(r['info'].n_diagrams) for r in runs)}), Yukawa lambda=1, r_s 1,2, "
                        f"beta E_F=25, {K} |k| in [0,3], VEGAS 50 bins, 2^{args.log2_samples} samples/iteration/order",
            "orders": orders, "n_k": K, "samples_per_iteration": N, "lambda_evaluated": 1, "rs": rs_list,
            "vegas_bins": 50,
        },
        "roofline": {
            "bound": "alu", "kernel": f"dmc_eval (order {dom['n']})", "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_unpacked_issue_rate": achieved / PEAK_ALU_TFLOPS,
            "traffic": traffic_for(dom["g"]) if dom["n"] == 3 and N == (1 << 24) else None,
            "kernel_ms": kern_ms, "flop_per_launch": fl_launch,
        },
    }
    if not args.no_peaks:
        out["peaks"] = measured_peaks()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(orders, K, args.cpu_seconds, beta, mu, lam, inst[0][3],
                                           workers=args.cpu_workers)
    last = dom["last"]
    j = int(np.argmin(np.abs(ks - 1.0)))
    out["estimate"] = {"order": dom["n"], "k": float(ks[j]), "re": float(last[0][0, 0, j].real),
                       "re_err": float(last[1][0, 0, j].real), "im": float(last[0][0, 0, j].imag),
                       "im_err": float(last[1][0, 0, j].imag)}
    if args.flow_order:
        out["flow_vs_vegas"] = flow_vs_vegas(args.flow_order, K, 1 << args.flow_log2_samples, args.flow_batches, beta, mu,
                                             lam, inst[0][3], train=args.flow_train, kind=args.flow_kind)
    if args.mcmc_orders:
        out["mcmc_vs_vegas"] = [mcmc_vs_vegas(int(n), beta, mu, lam, inst[0][3], n_chains=1 << args.mcmc_log2_chains,
                                              steps=args.mcmc_steps, thermal=args.mcmc_thermal,
                                              flow=not args.mcmc_no_flow, flow_kind=args.flow_kind,
                                              walk_every=args.mcmc_walk_every, walk_sigma=args.mcmc_walk_sigma)
                                for n in args.mcmc_orders.split(",")]
    if args.mass_order:
        out["effective_mass"] = effective_mass_leg(args.mass_order, args.mass_rs, args.mass_lambda, beta,
                                                   args.mass_log2_samples, args.mass_batches)
    if args.routing_orders:
        out["routing_compare"] = routing_compare([int(n) for n in args.routing_orders.split(",")])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
