// Host-side diagram front end and graph compiler (Sec. II: diagrams as computational graphs;
// Sec. V.A: front end, IR, back end).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace dmc {

constexpr int kMaxOrder = 6;
constexpr int kMaxTaylor = 6;  // highest total mu, lambda derivative order of a Taylor-mode graph

// A line of a routed diagram.  mom[j] (j < n) is the coefficient of loop momentum q_j and
// mom[n] the coefficient of the external k along the reference direction src -> dst.
struct Line {
    char kind;  // 'G' propagator, 'V' interaction
    int src, dst;
    std::array<int, kMaxOrder + 1> mom{};
};

struct Diagram {
    std::vector<int> sigma;  // propagator leaving vertex v enters sigma[v]
    int order = 0;
    int out_vertex = 0;      // sigma[out_vertex] == 0
    int n_fermion_loops = 0; // F
    double weight = 0;       // (-1)^(n+F) 2^F
    std::vector<Line> lines; // propagators (by source vertex, external skipped), then interactions
    int ext_line() const { return out_vertex / 2; }
};

// All connected, bridgeless (one-particle irreducible, tadpole free) self-energy diagrams of
// order n in canonical labelling, routed.
std::vector<Diagram> enumerate_sigma(int n);

// The canonical permutations of the order-n self-energies built bottom-up from the Dyson-Schwinger and parquet
// equations (every diagram exactly once, sorted); false with a message on an inconsistency.
bool construct_sigma(int n, std::vector<std::vector<int>>& out, std::string& err);

// The same diagram with its interaction lines and loop momenta taken from its building blocks
// (self-energy, dressed line, three- and four-point vertices, parquet channels); false with a
// message when the decomposition fails.
bool relabel_building_blocks(const Diagram& d, Diagram& out, std::string& err);

// ---- graph IR and code generation ----
enum class Op : uint8_t { Leaf, Mul, Fma, Add, MulC };

struct CodeStats {
    int64_t sample[4] = {0, 0, 0, 0};  // add, mul, fma, trans per sample (k-independent)
    int64_t k[4] = {0, 0, 0, 0};       // per (sample, k)
    int64_t k_deriv[4] = {0, 0, 0, 0}; // the part of k that only forms derivative roots
    int64_t naive[4] = {0, 0, 0, 0};   // plain sum of products per (sample, k)
    int parts = 1;                       // straight-line parts of the generated kernel
    int64_t sample_exec[4] = {0, 0, 0, 0};  // as executed by a kernel in parts (leaves recomputed
    int64_t k_exec[4] = {0, 0, 0, 0};       // per part); equal to sample / k for one part
    int64_t k_deriv_exec[4] = {0, 0, 0, 0};
};

struct Compiled {
    int order = 0, dim = 0, n_root_classes = 0;
    int n_momenta = 0, n_g_leaves = 0, n_v_leaves = 0, n_groups = 0;
    uint32_t deriv_mask = 0;
    int taylor_order = 0;  // 0: first-order tangents along the masked directions; T >= 1: Taylor mode
    int n_roots = 1;
    // per root, the coefficient it holds: d^m/dmu^m d^l/dlambda^l (d/dk)^e of the self-energy
    std::vector<std::array<int, 3>> root_orders;
    int part_size = 0;  // diagrams per straight-line part; 0 = one part
    int deriv_k = 0;    // derivative roots only at the first deriv_k external momenta (0: at all of them)
    int routing = 0;    // 0 path routing, 1 building-block variables
    int spin_deg = 2;   // factor per closed fermion loop
    int generation = 0; // 0 orderly enumeration, 1 bottom-up construction
    std::vector<Diagram> diagrams;
    CodeStats stats;
};

// Builds the compiled description (diagram subset selection, IR statistics).
// diagram_index < 0 keeps all diagrams.
// part_size: diagrams per straight-line part of the kernel; 0 chooses by size.
// taylor_order T >= 1 builds every derivative d^m/dmu^m d^l/dlambda^l with m + l <= T along the masked
// directions (mu bit 0, lambda bit 1), and with the k bit also the k derivative of each of them.
// routing 0: loop momenta on chords next to the external momentum's shortest path; 1: from the building
// blocks of the diagram (relabel_building_blocks), k on the shortest path.
// spin_deg: the factor of each closed fermion loop (2 for spin 1/2, 1 for spinless fermions).
// generation 0: the orderly enumeration; 1: the bottom-up construction (construct_sigma).
bool compile(int order, uint32_t deriv_mask, int taylor_order, int diagram_index, int part_size, int deriv_k,
             int routing, int spin_deg, int generation, Compiled& out, std::string& err);

// Device source for the evaluation kernel specialised to `n_groups` lambda groups.
std::string emit_eval_source(const Compiled& c, int n_groups, CodeStats* stats);

std::string export_text(const Compiled& c);

// Symbol of the generated kernel: order, lambda groups, roots.
std::string kernel_name(const Compiled& c, int n_groups);

}  // namespace dmc
