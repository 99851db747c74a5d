"""The bench's bookkeeping on the CPU: the C5 line's algorithmic FLOP from the graph's op counts, the flow
sampler's FLOP from its masks, and the traffic lookup keyed by the generated kernel source."""
import json
import os

import numpy as np

import functools

import bench
import paper_2403_18840_amd as dmc
import synth


@functools.lru_cache(maxsize=None)
def _c5_graph():
    return dmc.Graph(6, deriv_mask=dmc.D_K, deriv_k=1)


def test_affine_flow_flop_counts_the_networks_own_sizes():
    for D in (7, 15, 23):
        masks = synth.flow_masks(D, 8, 5)
        per = 0
        for m in masks:
            dA, dB = int(m.sum()), D - int(m.sum())
            per += 2 * (dA + 1) * 128      # first layer: the conditioning inputs and the bias input
            per += 2 * 128 * 128           # hidden layer
            per += 2 * 128 * 2 * dB        # s and t of the transformed dimensions
        assert bench.affine_flow_flop(masks) == per
        assert per < 8 * 2 * (16 * 128 + 128 * 128 + 128 * 32)   # below the padded tiles' count


def test_c5_flop_per_sample_and_group_from_op_counts():
    i = _c5_graph().info()
    K = 33
    per = (bench.flops(list(i.ops_sample)) + K * (bench.flops(list(i.ops_k)) - bench.flops(list(i.ops_k_deriv)))
           + bench.flops(list(i.ops_k_deriv)))
    assert per == 145243
    # the derivative-only part is evaluated at k_F alone: cheaper than the derivative at every momentum
    assert per < bench.flops(list(i.ops_sample)) + K * bench.flops(list(i.ops_k))


def test_traffic_lookup_is_keyed_by_the_kernel_source_and_launch_size():
    d = json.load(open(os.path.join(bench.ROOT, "profiles", "eval_o6_c5_hbm_traffic.json")))
    g = _c5_graph()
    assert bench.traffic_for(g, 3, 1 << 26, "eval_o6_c5_hbm_traffic.json") == d["hbm_bytes_per_launch"]
    assert bench.traffic_for(g, 3, 1 << 25, "eval_o6_c5_hbm_traffic.json") is None      # another launch size
    assert bench.traffic_for(g, 2, 1 << 26, "eval_o6_c5_hbm_traffic.json") is None      # another kernel
    assert bench.traffic_for(dmc.Graph(6), 3, 1 << 26, "eval_o6_c5_hbm_traffic.json") is None
    assert bench.traffic_for(g, 3, 1 << 26, "no_such_profile.json") is None
