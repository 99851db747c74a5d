"""Host-side checks of the C ABI library (no GPU): symbols, diagram export, errors, op counts."""
import math
import os
import re

import pytest

import paper_2403_18840_amd as dmc
from oracle import diagrams as dg

from golden_diagrams import golden_counts, golden_topologies, oracle_diagrams
from oracle import build as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "dmc.h")).read()
    declared = set(re.findall(r"\b(dmc_[a-z_0-9]+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = dmc.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} is declared in dmc.h but not exported"
    assert declared == set(dmc.ABI_SYMBOLS)


def _parse_export(text, n):
    out = set()
    for row in text.strip().splitlines():
        parts = [p.strip() for p in row.split("|")]
        sigma = tuple(int(t) for t in parts[0].split())
        w = float(parts[1].split()[1])
        ext = int(parts[2].split()[1])
        lines = []
        for part in parts[3:]:
            kind, *rest = part.split(None, 1)
            for seg in rest[0].split(";") if rest else []:
                v = [int(t) for t in seg.split()]
                if v:
                    lines.append((kind, v[0], v[1], tuple(v[2:])))
        out.add((sigma, w, ext, tuple(sorted(lines))))
    return out


def _oracle_set(n):
    out = set()
    for d in oracle_diagrams(n):
        lines = tuple(sorted((l.kind, l.src, l.dst, tuple(l.mom)) for l in d.lines))
        out.add((d.sigma, d.weight, d.ext_line, lines))
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_exported_diagrams_equal_oracle_set(n):
    # the library's orderly generator and the oracle's brute force give the same canonical
    # diagrams, the same signs and the same momentum routing (order 5 from the golden list that
    # the oracle's brute force wrote)
    g = dmc.Graph(n)
    assert _parse_export(g.export(), n) == _oracle_set(n)
    assert g.info().n_diagrams == len(oracle_diagrams(n))


@pytest.mark.parametrize("n,tops_expected", [(5, 2232), (6, 31130)])
def test_golden_counts(n, tops_expected):
    # each topology has (n-1)! 2^(n-1) labelled forms (the in-vertex's line is fixed)
    tops, lab = golden_counts(n)
    assert tops == tops_expected and lab == tops * math.factorial(n - 1) * 2 ** (n - 1)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_c_enumerator_matches_python_brute_force(n):
    # the C version of the oracle's brute force (used at order 6) against the Python one
    assert ob.enumerate_topologies(n) == dg.enumerate_topologies(n)


def test_c_enumerator_matches_order5_golden():
    tops, lab = ob.enumerate_topologies(5)
    assert tops == golden_topologies(5) and lab == golden_counts(5)[1]


def test_partitioned_graphs():
    # large graphs are emitted as several straight-line parts that share nothing
    for n, mask, parts in [(3, 0, 1), (4, 0, 1), (4, 7, 1), (5, 0, 1), (5, 7, 3), (6, 0, 13)]:
        i = dmc.Graph(n, deriv_mask=mask).info()
        assert i.n_parts == parts, (n, mask, i.n_parts)
    g = dmc.Graph(4, part_size=40)
    i = g.info()
    assert i.n_parts == 5 and i.part_size == 40
    src = g.source(1)
    assert "_p5" in src and src.count("// part ") == 5
    assert src.count("__attribute__((noinline)) void dmc_part_") == 5 and "dmc_part_4(&a, (const LdsF*)cin, (LdsF*)(stage + lane), (const LdsF*)kl_s, kb, nkc, grp, ml);" in src
    # the parts read the momenta from the block's LDS copy; a device function has no kernel-argument pointer
    # of its own (the compiler gives it a null base), so the parts must never ask for one
    assert src.count("const float kk = kl[ki];") == 5 and "kernarg_segment_ptr" not in src
    assert src.count("__builtin_amdgcn_readfirstlane(kb_)") == 5
    # every diagram lands in exactly one part
    import re
    sizes = [int(m) for m in re.findall(r"// part \d+ \((\d+) diagrams\)", src)]
    assert sum(sizes) == 189 and max(sizes) == 40
    # splitting costs extra leaf evaluations (executed counts) but not algorithmic ones
    assert list(i.ops_k) == list(dmc.Graph(4).info().ops_k)
    assert sum(i.ops_k_exec) > sum(i.ops_k) and i.ops_k_exec[3] > i.ops_k[3]
    with pytest.raises(dmc.DmcError):
        dmc.Graph(3, part_size=-1)


def test_single_diagram_graph_and_errors():
    g = dmc.Graph(3, diagram_index=5)
    assert g.info().n_diagrams == 1
    for bad in [dict(order=0), dict(order=7), dict(order=2, diagram_index=99), dict(order=2, deriv_mask=8)]:
        with pytest.raises(dmc.DmcError) as e:
            dmc.Graph(**bad)
        assert e.value.status == -1


def test_compaction_reduces_operation_count():
    # the factored graph executes far fewer operations per (sample, k) than the plain sum
    for n, factor in [(3, 5), (4, 20)]:
        i = dmc.Graph(n).info()
        assert sum(i.ops_naive) > factor * (sum(i.ops_k))


def _k_loop(src):
    a = src.index("const float kk = a.k[ki];")
    return src[a:src.index("const float FR0_0", a)]


def test_factoring_keeps_multipliers_out_of_the_momentum_loop():
    # hoisted multipliers (propagator signs, k-independent factors, constants) are applied outside the loop
    # over external momenta: no sign select, no lambda add and no mu subtraction inside it, and the sample's
    # Jacobian sits in the per-sample phase factors; issue slots per (sample, k) (transcendentals twice)
    # stay at or below the factored counts
    for n, most in [(2, 27), (3, 62), (4, 140)]:
        g = dmc.Graph(n)
        src = g.source(1)
        loop = _k_loop(src)
        assert " ? -" not in loop and "+ LAM0" not in loop and "MU - " not in loop
        assert " * J;" in src[:src.index("const float kk = a.k[ki];")]
        i = g.info()
        assert sum(i.ops_k) + i.ops_k[3] <= most, (n, list(i.ops_k))


def test_generated_source_mentions_every_group():
    src = dmc.Graph(2).source(3)
    assert "LAM2" in src and "#define NGRP 3" in src


def test_accumulator_and_sampler_argument_errors():
    for args in [(0, 4, 1), (1, 0, 1), (1, 65, 1), (9, 4, 1), (1, 4, 5)]:
        with pytest.raises(dmc.DmcError):
            dmc.Accumulator(*args)
    for args in [(5, 2), (1, 9), (1, 0)]:
        with pytest.raises(dmc.DmcError):
            dmc.Sampler(*args)
    with pytest.raises(dmc.DmcError):
        dmc.Sampler(dmc.SAMPLER_VEGAS, 2, n_bins=500)


def test_host_vegas_refine_matches_oracle():
    # the library's FP64 refinement (host code; the sampler applies it to its gathered histogram) against the
    # oracle's, on histograms spanning many decades with empty and tiny bins, and an already adapted grid
    import numpy as np
    from oracle import sampler as osp
    import synth
    rng = np.random.default_rng(4)
    for D, B, alpha in ((3, 50, 0.5), (7, 50, 1.0), (11, 20, 0.0), (2, 2, 0.5)):
        edges = synth.vegas_grid(D, B, seed=D).astype(np.float64) if B == 50 else \
            np.tile(np.linspace(0.0, 1.0, B + 1), (D, 1))
        h = 10.0 ** rng.uniform(-80, 3, size=(D, B))
        h[rng.random((D, B)) < 0.2] = 0.0
        got = dmc.vegas_refine(edges, h, alpha)
        want = osp.refine_grid(edges, h, alpha)
        assert np.allclose(got, want, rtol=0, atol=1e-12), (D, B, alpha, np.abs(got - want).max())
    with pytest.raises(dmc.DmcError):
        dmc.vegas_refine(np.zeros((2, 3)), np.zeros((2, 2)), -1.0)


def test_spin_degeneracy_weights():
    """spec.spin_deg: 2 (and 0) gives (-1)^(n+F) 2^F, 1 gives the spinless (-1)^(n+F); other values are refused."""
    for n in (2, 3, 4):
        two = _parse_export(dmc.Graph(n).export(), n)
        assert two == _parse_export(dmc.Graph(n, spin_deg=0).export(), n)
        one = _parse_export(dmc.Graph(n, spin_deg=1).export(), n)
        assert dmc.Graph(n, spin_deg=0).info().spin_deg == 2 and dmc.Graph(n, spin_deg=1).info().spin_deg == 1
        loops = {d.sigma: d.n_loops_f for d in oracle_diagrams(n)}
        assert {(s, (-1.0) ** (n + loops[s]), e, l) for s, w, e, l in two} == {(s, w / 2.0 ** loops[s], e, l) for s, w, e, l in two}
        assert one == {(s, (-1.0) ** (n + loops[s]), e, l) for s, w, e, l in two}
    with pytest.raises(dmc.DmcError):
        dmc.Graph(2, spin_deg=3)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_bottom_up_construction_equals_enumeration(n):
    """spec.generation = DMC_GENERATE_CONSTRUCT: the library's Dyson-Schwinger/parquet construction gives the same
    diagrams, signs and routing as its orderly enumeration (and so as the oracle's brute force)."""
    g = dmc.Graph(n, generation=dmc.GENERATE_CONSTRUCT)
    assert g.info().generation == 1 and g.info().n_diagrams == len(oracle_diagrams(n))
    assert _parse_export(g.export(), n) == _parse_export(dmc.Graph(n).export(), n)
    if n == 2:
        with pytest.raises(dmc.DmcError):
            dmc.Graph(2, generation=2)


def test_constructed_graph_compiles_to_the_same_kernel():
    """The graph builder does not depend on the order of the diagram list: the bottom-up construction's graph emits
    the same kernel source as the enumeration's."""
    for n in (3, 5):
        assert dmc.Graph(n, generation=dmc.GENERATE_CONSTRUCT).source(1) == dmc.Graph(n).source(1)
