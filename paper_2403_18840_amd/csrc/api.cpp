// C ABI of the library (declared in include/dmc.h): handles, run-time compilation of the graph
// kernels, launches, the FP64 estimate and the VEGAS grid refinement.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dmc.h"
#include "graph.hpp"
#include "flow.hpp"
#include "kernels.hpp"
#include "mcmc.hpp"
#include "nsf.hpp"
#include "probe.hpp"

namespace {

thread_local std::string g_err;

dmc_status fail(dmc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

}  // namespace

namespace dmc {
// the thread-local error text for the other translation units of the library
dmc_status set_error(dmc_status s, const char* msg) { return fail(s, msg); }
}  // namespace dmc

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(DMC_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

#define HIP_ALLOC(expr)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)                             \
            return fail(DMC_E_NOMEM, std::string(#expr ": ") + hipGetErrorString(e_));               \
        if (e_ != hipSuccess) return fail(DMC_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

hipStream_t S(void* p) { return reinterpret_cast<hipStream_t>(p); }

int cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int max_blocks_per_cu = 1;
    std::string src;
    // kernels in parts: the chunk of external momenta staged per pass and the blocks per CU it allows,
    // by the number of external momenta (0: not chosen yet)
    int kc[65] = {0};
    int kc_blocks[65] = {0};
};

// the EvalArgs layout the generated kernel declares
struct EvalArgs {
    const float* x;
    long long ld;
    const float* jac;
    long long n;
    double* partial;
    unsigned int* nonfinite;
    float* f_out;
    float* imp_out;
    int n_k, s_total, kc, imp_roots;
    float mu, beta, bl, blmu, inv2beta, pad2;
    float lam[8];
    float scale[8];
    float k[64];
};

}  // namespace

struct dmc_graph {
    dmc::Compiled c;
    std::map<std::pair<int, int>, JitKernel> jit;  // (device, n_groups)
    std::string exported;
    int imp_roots = 1;  // leading roots whose |w| make up the importance (imp_out)
};

struct dmc_accum {
    int n_groups, n_k, n_roots, s_total;
    double* totals = nullptr;                  // device [s_total][2]
    unsigned long long* nonfin_tot = nullptr;  // device
    double* partial = nullptr;                 // device [cap_blocks][s_total][2]
    unsigned int* nonfin_part = nullptr;       // device [cap_blocks]
    int cap_blocks = 0;
    int pending_blocks = 0;
    int64_t pending_n = 0;
    int64_t n_samples = 0;
    // instances of the last eval_batch: group and factor (gamma / gamma_group)^n
    std::vector<int> inst_group;
    std::vector<double> inst_factor;
};

struct dmc_sampler {
    int kind, order, dim, n_bins;
    double beta, qmax;
    std::vector<double> edges;  // host [dim][n_bins + 1]
    float* d_edges = nullptr;
    double* d_hist = nullptr;               // [dim][n_bins]
    unsigned long long* d_hist_u = nullptr;  // [dim][n_bins]
    unsigned int* d_max = nullptr;
    uint64_t last_seed = 0, last_first = 0;
    int64_t last_n = -1;
};

extern "C" {

const char* dmc_last_error(void) { return g_err.c_str(); }
const char* dmc_version(void) { return "dmc-mi355x 0.1 (gfx950)"; }

// ------------------------------------------------------------------------------ graph
dmc_status dmc_compile_graph(const dmc_graph_spec* spec, dmc_graph** out) {
    if (!spec || !out) return fail(DMC_E_INVALID, "null argument");
    if (spec->part_size < 0) return fail(DMC_E_INVALID, "part_size must be >= 0");
    auto g = std::make_unique<dmc_graph>();
    std::string err;
    try {
        if (!dmc::compile(spec->order, spec->deriv_mask, spec->taylor_order, spec->diagram_index, spec->part_size,
                          spec->deriv_k, spec->routing, spec->spin_deg == 0 ? 2 : spec->spin_deg, spec->generation,
                          g->c, err))
            return fail(DMC_E_INVALID, err);
        g->exported = dmc::export_text(g->c);
    } catch (const std::bad_alloc&) {
        return fail(DMC_E_NOMEM, "host allocation failed");
    }
    *out = g.release();
    return DMC_OK;
}

dmc_status dmc_graph_set_importance(dmc_graph* g, int32_t n_roots) {
    if (!g) return fail(DMC_E_INVALID, "null graph");
    if (n_roots < 1 || n_roots > g->c.n_roots) return fail(DMC_E_INVALID, "need 1 <= n_roots <= the graph's roots");
    g->imp_roots = n_roots;
    return DMC_OK;
}

dmc_status dmc_graph_query(const dmc_graph* g, dmc_graph_info* o) {
    if (!g || !o) return fail(DMC_E_INVALID, "null argument");
    std::memset(o, 0, sizeof(*o));
    o->order = g->c.order;
    o->dim = g->c.dim;
    o->n_diagrams = (int)g->c.diagrams.size();
    o->n_root_classes = g->c.n_root_classes;
    o->n_parts = g->c.stats.parts;
    o->part_size = g->c.part_size;
    for (int i = 0; i < 4; ++i) {
        o->ops_sample[i] = g->c.stats.sample[i];
        o->ops_k[i] = g->c.stats.k[i];
        o->ops_naive[i] = g->c.stats.naive[i];
        o->ops_sample_exec[i] = g->c.stats.sample_exec[i];
        o->ops_k_exec[i] = g->c.stats.k_exec[i];
        o->ops_k_deriv[i] = g->c.stats.k_deriv[i];
        o->ops_k_deriv_exec[i] = g->c.stats.k_deriv_exec[i];
    }
    o->n_roots = g->c.n_roots;
    o->taylor_order = g->c.taylor_order;
    o->deriv_k = g->c.deriv_k;
    o->routing = g->c.routing;
    o->spin_deg = g->c.spin_deg;
    o->generation = g->c.generation;
    return DMC_OK;
}

dmc_status dmc_graph_root_orders(const dmc_graph* g, int32_t* out, int32_t cap) {
    if (!g || !out) return fail(DMC_E_INVALID, "null argument");
    if (cap < 3 * g->c.n_roots) return fail(DMC_E_INVALID, "cap must be at least 3 n_roots");
    for (int r = 0; r < g->c.n_roots; ++r)
        for (int i = 0; i < 3; ++i) out[3 * r + i] = g->c.root_orders[r][i];
    return DMC_OK;
}

static dmc_status copy_text(const std::string& t, char* buf, size_t cap, size_t* len) {
    if (len) *len = t.size();
    if (!buf) return DMC_OK;
    if (cap < t.size() + 1) return fail(DMC_E_INVALID, "buffer too small");
    std::memcpy(buf, t.c_str(), t.size() + 1);
    return DMC_OK;
}

dmc_status dmc_graph_export_diagrams(const dmc_graph* g, char* buf, size_t cap, size_t* len) {
    if (!g) return fail(DMC_E_INVALID, "null graph");
    return copy_text(g->exported, buf, cap, len);
}

dmc_status dmc_graph_source(const dmc_graph* g, int32_t n_groups, char* buf, size_t cap, size_t* len) {
    if (!g || n_groups < 1 || n_groups > DMC_MAX_GROUPS) return fail(DMC_E_INVALID, "bad graph or n_groups");
    return copy_text(dmc::emit_eval_source(g->c, n_groups, nullptr), buf, cap, len);
}

void dmc_graph_destroy(dmc_graph* g) {
    if (!g) return;
    for (auto& kv : g->jit)
        if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
    delete g;
}

// On-disk cache of compiled graph kernels: an order-6 graph takes tens of seconds of run-time
// compilation.  Directory: $DMC_KERNEL_CACHE (empty: no cache), else $XDG_CACHE_HOME/dmc-kernels,
// else $HOME/.cache/dmc-kernels.  Key: 64-bit FNV-1a of compiler version, options and source.
static std::string cache_dir() {
    const char* e = std::getenv("DMC_KERNEL_CACHE");
    if (e) return std::string(e);
    if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/dmc-kernels";
    if (const char* h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/dmc-kernels";
    return std::string();
}

static uint64_t fnv1a(const std::string& t, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : t) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

static bool read_file(const std::string& path, std::vector<char>& out) {
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long sz = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    out.resize(sz > 0 ? (size_t)sz : 0);
    const bool ok = sz > 0 && std::fread(out.data(), 1, out.size(), f) == out.size();
    std::fclose(f);
    return ok;
}

static void write_file_atomic(const std::string& dir, const std::string& name, const std::vector<char>& data) {
    std::error_code ec;
    std::filesystem::create_directories(dir, ec);
    if (ec) return;
    const std::string tmp = dir + "/" + name + ".tmp" + std::to_string((long long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    std::fclose(f);
    if (ok)
        std::filesystem::rename(tmp, dir + "/" + name, ec);
    else
        std::filesystem::remove(tmp, ec);
}

static dmc_status get_kernel(dmc_graph* g, int n_groups, JitKernel** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_pair(dev, n_groups);
    auto it = g->jit.find(key);
    if (it != g->jit.end()) {
        *out = &it->second;
        return DMC_OK;
    }
    JitKernel jk;
    jk.src = dmc::emit_eval_source(g->c, n_groups, nullptr);
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    int vmaj = 0, vmin = 0;
    hiprtcVersion(&vmaj, &vmin);
    std::string tag = "hiprtc " + std::to_string(vmaj) + "." + std::to_string(vmin);
    for (const char* o : opts) tag += std::string(" ") + o;
    char hex[17];
    std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)fnv1a(jk.src, fnv1a(tag)));
    const std::string cdir = cache_dir(), cname = std::string(hex) + ".co";
    std::vector<char> cached;
    if (!cdir.empty() && read_file(cdir + "/" + cname, cached) &&
        hipModuleLoadData(&jk.mod, cached.data()) == hipSuccess) {
        HIP_TRY(hipModuleGetFunction(&jk.fn, jk.mod, dmc::kernel_name(g->c, n_groups).c_str()));
        g->jit[key] = jk;
        *out = &g->jit[key];
        return DMC_OK;
    }
    (void)hipGetLastError();  // a stale cache entry that failed to load is recompiled
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, jk.src.c_str(), "dmc_eval.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(DMC_E_COMPILE, "hiprtcCreateProgram failed");
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(DMC_E_COMPILE, "graph kernel compilation failed: " + log);
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    HIP_TRY(hipModuleLoadData(&jk.mod, code.data()));
    if (!cdir.empty()) write_file_atomic(cdir, cname, code);
    HIP_TRY(hipModuleGetFunction(&jk.fn, jk.mod, dmc::kernel_name(g->c, n_groups).c_str()));
    g->jit[key] = jk;
    *out = &g->jit[key];
    return DMC_OK;
}

// ------------------------------------------------------------------------------ accumulator
dmc_status dmc_accum_create(int32_t n_groups, int32_t n_k, int32_t n_roots, dmc_accum** out) {
    if (!out || n_groups < 1 || n_groups > DMC_MAX_GROUPS || n_k < 1 || n_k > DMC_MAX_K || n_roots < 1 ||
        n_roots > DMC_MAX_ROOTS)
        return fail(DMC_E_INVALID, "accumulator shape out of range");
    auto a = std::make_unique<dmc_accum>();
    a->inst_group.reserve(DMC_MAX_INSTANCES);
    a->inst_factor.reserve(DMC_MAX_INSTANCES);
    a->n_groups = n_groups;
    a->n_k = n_k;
    a->n_roots = n_roots;
    a->s_total = n_k * 2 * n_groups * n_roots;
    HIP_ALLOC(hipMalloc(&a->totals, sizeof(double) * 2 * a->s_total));
    HIP_ALLOC(hipMalloc(&a->nonfin_tot, sizeof(unsigned long long)));
    HIP_TRY(hipMemset(a->totals, 0, sizeof(double) * 2 * a->s_total));
    HIP_TRY(hipMemset(a->nonfin_tot, 0, sizeof(unsigned long long)));
    *out = a.release();
    return DMC_OK;
}

dmc_status dmc_accum_reset(dmc_accum* a, void* stream) {
    if (!a) return fail(DMC_E_INVALID, "null accumulator");
    HIP_TRY(hipMemsetAsync(a->totals, 0, sizeof(double) * 2 * a->s_total, S(stream)));
    HIP_TRY(hipMemsetAsync(a->nonfin_tot, 0, sizeof(unsigned long long), S(stream)));
    a->n_samples = 0;
    a->pending_blocks = 0;
    a->pending_n = 0;
    return DMC_OK;
}

void dmc_accum_destroy(dmc_accum* a) {
    if (!a) return;
    (void)hipFree(a->totals);
    (void)hipFree(a->nonfin_tot);
    (void)hipFree(a->partial);
    (void)hipFree(a->nonfin_part);
    delete a;
}

// ------------------------------------------------------------------------------ evaluation
// The evaluation launch shared by dmc_eval_batch and the allocation-free entry point.  With `fixed`
// (a device buffer of fixed_bytes for the block partials and non-finite counts) nothing is
// allocated: the kernel must already be loaded, the block count is capped by the buffer, and the
// partials are folded into the accumulator right away.
static dmc_status eval_launch(dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext, int32_t n_k,
                              const float* x, int64_t ld, const float* jac, int64_t n, dmc_accum* acc, float* f_out,
                              float* imp_out, void* stream, void* fixed, size_t fixed_bytes) {
    if (!g || !inst || !k_ext || !x || !jac || !acc) return fail(DMC_E_INVALID, "null argument");
    if (n_inst < 1 || n_inst > DMC_MAX_INSTANCES) return fail(DMC_E_INVALID, "n_inst out of range");
    if (n_k < 1 || n_k > DMC_MAX_K) return fail(DMC_E_INVALID, "n_k out of range");
    if (n < 1 || ld < n) return fail(DMC_E_INVALID, "need n >= 1 and ld >= n");
    if (acc->pending_blocks) return fail(DMC_E_STATE, "dmc_accumulate must follow each dmc_eval_batch");
    const double beta = inst[0].beta, mu = inst[0].mu;
    if (!(beta > 0) || !(beta * std::fabs(mu) < 80.0)) return fail(DMC_E_INVALID, "need beta > 0, beta |mu| < 80");
    // lambda groups (fixed-size arrays: no allocation)
    double lam[DMC_MAX_GROUPS], gam[DMC_MAX_GROUPS];
    int grp[DMC_MAX_INSTANCES];
    double fac[DMC_MAX_INSTANCES];
    int ng = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (inst[i].beta != beta || inst[i].mu != mu) return fail(DMC_E_INVALID, "instances must share beta and mu");
        if (!(inst[i].lambda > 0) || !(inst[i].gamma > 0)) return fail(DMC_E_INVALID, "need lambda > 0, gamma > 0");
        int gi = -1;
        for (int j = 0; j < ng; ++j)
            if (lam[j] == inst[i].lambda) gi = j;
        if (gi < 0) {
            if (ng == DMC_MAX_GROUPS) return fail(DMC_E_INVALID, "too many distinct lambda values");
            gi = ng++;
            lam[gi] = inst[i].lambda;
            gam[gi] = inst[i].gamma;
        }
        grp[i] = gi;
        fac[i] = std::pow(inst[i].gamma / gam[gi], g->c.order);
    }
    if (ng != acc->n_groups || n_k != acc->n_k || g->c.n_roots != acc->n_roots)
        return fail(DMC_E_INVALID, "accumulator shape does not match graph, lambda groups and n_k");
    JitKernel* jk = nullptr;
    if (fixed) {
        // the allocation-free path never compiles or loads a module
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        auto it = g->jit.find(std::make_pair(dev, ng));
        if (it == g->jit.end())
            return fail(DMC_E_STATE, "the graph's kernel for this many lambda groups is not loaded on this device yet "
                                     "(one dmc_eval_batch call loads it)");
        jk = &it->second;
    } else {
        dmc_status st = get_kernel(g, ng, &jk);
        if (st != DMC_OK) return st;
    }

    const int NR = g->c.n_roots;
    const bool split = g->c.stats.parts > 1;
    // LDS per block of four waves: the stage, the FP64 totals and, for a kernel in parts, the lanes' inputs
    // (3n + 2(n - 1) rows per wave).  A single-part kernel stages KC momenta of every group (fixed at
    // compile time); a kernel in parts stages kc momenta of one group, kc chosen here: the largest chunk
    // that keeps the blocks per CU its registers allow (each extra chunk reruns the parts' k-independent
    // code), else the chunk with the most blocks per CU
    const int nin = split ? 3 * g->c.order + 2 * (g->c.order - 1) : 0;
    auto smem_for = [&](int stage_floats) {
        return (size_t)4 * stage_floats * 64 * sizeof(float) + (size_t)4 * 2 * acc->s_total * sizeof(double) +
               (size_t)4 * nin * 64 * sizeof(float);
    };
    auto blocks_for = [&](size_t smem) {
        int nb = 0;
        if (smem > 160 * 1024 ||
            hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, jk->fn, 256, smem) != hipSuccess)
            return 0;
        return nb;
    };
    int kc = 0;
    size_t smem = 0;
    if (!split) {
        const int SPK = 2 * ng * NR;
        const int KC = SPK <= 16 ? 16 / SPK : 1;
        smem = smem_for(16 * ((KC * SPK + 15) / 16));
        if (smem > 160 * 1024) return fail(DMC_E_INVALID, "too many accumulator slots for one workgroup");
        if (jk->max_blocks_per_cu <= 1) {
            const int nb = blocks_for(smem);
            if (nb > 0) jk->max_blocks_per_cu = nb;
        }
    } else {
        // staged floats per lane for a chunk of c momenta: 2 NR for each of the first momenta that carry
        // derivative roots (spec.deriv_k; all of them when 0), 2 for the others.  The chunk holds at
        // least the derivative momenta, so that they all fall into the first chunk.
        const int KD = NR > 1 ? g->c.deriv_k : 0;
        auto stage_for = [&](int c) {
            const int ml = KD ? std::min(KD, c) : c;
            return ml * 2 * NR + (c - ml) * 2;
        };
        const int cmin = KD ? std::min(KD, n_k) : 1;
        if (!jk->kc[n_k]) {
            const int best = blocks_for(smem_for(stage_for(cmin)));
            if (best < 1) return fail(DMC_E_INVALID, "too many accumulator slots for one workgroup");
            int pick = cmin, pick_nb = best;
            for (int c = n_k; c >= cmin; --c) {
                const int nb = blocks_for(smem_for(stage_for(c)));
                if (nb >= best) {
                    pick = c;
                    pick_nb = nb;
                    break;
                }
            }
            jk->kc[n_k] = pick;
            jk->kc_blocks[n_k] = pick_nb;
        }
        kc = jk->kc[n_k];
        smem = smem_for(stage_for(kc));
        jk->max_blocks_per_cu = jk->kc_blocks[n_k];
    }
    const int64_t ntiles = (n + 255) / 256;
    int64_t cap = (int64_t)cu_count() * std::min(jk->max_blocks_per_cu, 8);
    double* partial = acc->partial;
    unsigned int* nonfin_part = acc->nonfin_part;
    if (fixed) {
        // per block: 2 s_total FP64 partial sums and one non-finite count
        const size_t per = sizeof(double) * 2 * (size_t)acc->s_total + sizeof(unsigned int);
        const int64_t fit = (int64_t)(fixed_bytes / per);
        if (fit < 1) return fail(DMC_E_INVALID, "the accumulator's slots exceed the static scratch of one block");
        cap = std::min(cap, fit);
    }
    const int nb = (int)std::min<int64_t>(ntiles, cap);
    if (fixed) {
        partial = static_cast<double*>(fixed);
        nonfin_part = reinterpret_cast<unsigned int*>(partial + (size_t)2 * acc->s_total * nb);
    } else if (nb > acc->cap_blocks) {
        (void)hipFree(acc->partial);
        (void)hipFree(acc->nonfin_part);
        acc->partial = nullptr;
        acc->nonfin_part = nullptr;
        acc->cap_blocks = 0;
        HIP_ALLOC(hipMalloc(&acc->partial, sizeof(double) * 2 * acc->s_total * (size_t)nb));
        HIP_ALLOC(hipMalloc(&acc->nonfin_part, sizeof(unsigned int) * (size_t)nb));
        acc->cap_blocks = nb;
        partial = acc->partial;
        nonfin_part = acc->nonfin_part;
    }
    EvalArgs a;
    std::memset(&a, 0, sizeof(a));
    a.x = x;
    a.ld = ld;
    a.jac = jac;
    a.n = n;
    a.partial = partial;
    a.nonfinite = nonfin_part;
    a.f_out = f_out;
    a.imp_out = imp_out;
    a.n_k = n_k;
    a.s_total = acc->s_total;
    a.kc = kc;
    a.imp_roots = g->imp_roots;
    a.mu = (float)mu;
    a.beta = (float)beta;
    a.bl = (float)(beta * M_LOG2E);
    a.blmu = (float)(beta * M_LOG2E * mu);
    a.inv2beta = (float)(0.5 / beta);
    const int nord = g->c.order;
    for (int gi = 0; gi < ng; ++gi) {
        a.lam[gi] = (float)lam[gi];
        // (8 pi gamma)^n (2 pi)^(-3n): the interaction strength and loop measure, applied once
        a.scale[gi] = (float)(std::pow(8.0 * M_PI * gam[gi], nord) * std::pow(2.0 * M_PI, -3.0 * nord));
    }
    for (int j = 0; j < n_k; ++j) a.k[j] = k_ext[j];
    void* params[] = {&a};
    HIP_TRY(hipModuleLaunchKernel(jk->fn, nb, 1, 1, 256, 1, 1, (unsigned)smem, S(stream), params, nullptr));
    // the accumulator's instance vectors hold DMC_MAX_INSTANCES entries of capacity: assign does not allocate
    acc->inst_group.assign(grp, grp + n_inst);
    acc->inst_factor.assign(fac, fac + n_inst);
    if (fixed) {
        HIP_TRY(dmc::launch_fold(partial, nb, 2 * acc->s_total, acc->totals, nonfin_part, acc->nonfin_tot, S(stream)));
        acc->n_samples += n;
        return DMC_OK;
    }
    acc->pending_blocks = nb;
    acc->pending_n = n;
    return DMC_OK;
}

dmc_status dmc_eval_batch(dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext, int32_t n_k,
                          const float* x, int64_t ld, const float* jac, int64_t n, dmc_accum* acc, float* f_out,
                          float* imp_out, void* stream) {
    return eval_launch(g, inst, n_inst, k_ext, n_k, x, ld, jac, n, acc, f_out, imp_out, stream, nullptr, 0);
}

// The static device scratch (kernels.hip) as a device address, per device, taken once with that device
// current: in host code the array's name is not a device address.
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {nullptr};

dmc_status dmc_eval_accumulate_noalloc(dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext,
                                       int32_t n_k, const float* x, int64_t ld, const float* jac, int64_t n,
                                       dmc_accum* acc, float* f_out, float* imp_out, void* stream) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(DMC_E_DEVICE, "device index out of range for the static scratch");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            HIP_TRY(dmc::scratch_address(&p));
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    return eval_launch(g, inst, n_inst, k_ext, n_k, x, ld, jac, n, acc, f_out, imp_out, stream, ptr,
                       dmc::kScratchBytes);
}

dmc_status dmc_accumulate(dmc_accum* acc, dmc_sampler* s, const float* imp, void* stream) {
    if (!acc) return fail(DMC_E_INVALID, "null accumulator");
    if (!acc->pending_blocks) return fail(DMC_E_STATE, "no dmc_eval_batch to fold");
    if (s && s->kind == DMC_SAMPLER_VEGAS) {
        if (!imp) return fail(DMC_E_INVALID, "the VEGAS histogram needs the importance buffer");
        if (s->last_n != acc->pending_n) return fail(DMC_E_STATE, "sampler's last batch does not match the evaluation");
    }
    HIP_TRY(dmc::launch_fold(acc->partial, acc->pending_blocks, 2 * acc->s_total, acc->totals, acc->nonfin_part,
                             acc->nonfin_tot, S(stream)));
    acc->n_samples += acc->pending_n;
    acc->pending_blocks = 0;
    if (s && s->kind == DMC_SAMPLER_VEGAS) {
        dmc::HistArgs h;
        h.imp = imp;
        h.n = s->last_n;
        h.seed = s->last_seed;
        h.first = s->last_first;
        h.dim = s->dim;
        h.n_bins = s->n_bins;
        h.maxbits = s->d_max;
        h.hist_u64 = s->d_hist_u;
        h.hist = s->d_hist;
        HIP_TRY(dmc::launch_hist(h, cu_count(), S(stream)));
    }
    return DMC_OK;
}

dmc_status dmc_accum_read(dmc_accum* acc, double* sums, int64_t* n_samples, void* stream) {
    if (!acc || !sums) return fail(DMC_E_INVALID, "null argument");
    std::vector<double> t(2 * acc->s_total);
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipMemcpy(t.data(), acc->totals, sizeof(double) * t.size(), hipMemcpyDeviceToHost));
    // device slot order [k][group][root][comp] -> [group][root][k][comp]
    const int NG = acc->n_groups, NR = acc->n_roots, K = acc->n_k;
    for (int g = 0; g < NG; ++g)
        for (int r = 0; r < NR; ++r)
            for (int k = 0; k < K; ++k)
                for (int c = 0; c < 2; ++c) {
                    const int gs = k * (2 * NG * NR) + (g * NR + r) * 2 + c;
                    const size_t o = ((((size_t)g * NR + r) * K + k) * 2 + c) * 2;
                    sums[o] = t[2 * gs];
                    sums[o + 1] = t[2 * gs + 1];
                }
    if (n_samples) *n_samples = acc->n_samples;
    return DMC_OK;
}

dmc_status dmc_estimate(dmc_accum* acc, double* mean, double* stderr_, int64_t* n_samples, int64_t* n_nonfinite,
                        void* stream) {
    if (!acc || !mean || !stderr_) return fail(DMC_E_INVALID, "null argument");
    if (acc->inst_group.empty()) return fail(DMC_E_STATE, "no evaluation yet");
    const int NG = acc->n_groups, NR = acc->n_roots, K = acc->n_k;
    std::vector<double> sums((size_t)NG * NR * K * 4);
    dmc_status st = dmc_accum_read(acc, sums.data(), nullptr, stream);
    if (st != DMC_OK) return st;
    unsigned long long nf = 0;
    HIP_TRY(hipMemcpy(&nf, acc->nonfin_tot, sizeof(nf), hipMemcpyDeviceToHost));
    const double N = (double)acc->n_samples;
    for (size_t i = 0; i < acc->inst_group.size(); ++i) {
        const int g = acc->inst_group[i];
        const double f = acc->inst_factor[i];
        for (int r = 0; r < NR; ++r)
            for (int k = 0; k < K; ++k)
                for (int c = 0; c < 2; ++c) {
                    const size_t o = ((((size_t)g * NR + r) * K + k) * 2 + c) * 2;
                    const double m = sums[o] / N;
                    const double var = N > 1 ? std::max(0.0, (sums[o + 1] / N - m * m)) / (N - 1) : 0.0;
                    const size_t oi = (((size_t)i * NR + r) * K + k) * 2 + c;
                    mean[oi] = f * m;
                    stderr_[oi] = f * std::sqrt(var);
                }
    }
    if (n_samples) *n_samples = acc->n_samples;
    if (n_nonfinite) *n_nonfinite = (int64_t)nf;
    return nf ? fail(DMC_E_NUMERIC, "non-finite sample weights were dropped") : DMC_OK;
}

// ------------------------------------------------------------------------------ sampler
dmc_status dmc_sampler_create(int32_t kind, int32_t order, int32_t n_bins, double beta, double qmax,
                              dmc_sampler** out) {
    if (!out) return fail(DMC_E_INVALID, "null out");
    if (kind != DMC_SAMPLER_UNIFORM && kind != DMC_SAMPLER_VEGAS) return fail(DMC_E_INVALID, "unknown sampler kind");
    if (order < 1 || order > DMC_MAX_ORDER) return fail(DMC_E_INVALID, "order out of range");
    if (kind == DMC_SAMPLER_VEGAS && (n_bins < 2 || n_bins > 128)) return fail(DMC_E_INVALID, "n_bins in 2..128");
    if (!(beta > 0) || !(qmax > 0)) return fail(DMC_E_INVALID, "need beta > 0 and qmax > 0");
    auto s = std::make_unique<dmc_sampler>();
    s->kind = kind;
    s->order = order;
    s->dim = 4 * order - 1;
    s->n_bins = kind == DMC_SAMPLER_VEGAS ? n_bins : 1;
    s->beta = beta;
    s->qmax = qmax;
    const int B = s->n_bins;
    s->edges.resize((size_t)s->dim * (B + 1));
    for (int d = 0; d < s->dim; ++d)
        for (int b = 0; b <= B; ++b) s->edges[(size_t)d * (B + 1) + b] = (double)b / B;
    const size_t nc = (size_t)s->dim * B;
    HIP_ALLOC(hipMalloc(&s->d_edges, sizeof(float) * s->edges.size()));
    HIP_ALLOC(hipMalloc(&s->d_hist, sizeof(double) * nc));
    HIP_ALLOC(hipMalloc(&s->d_hist_u, sizeof(unsigned long long) * nc));
    HIP_ALLOC(hipMalloc(&s->d_max, sizeof(unsigned int)));
    std::vector<float> ef(s->edges.begin(), s->edges.end());
    HIP_TRY(hipMemcpy(s->d_edges, ef.data(), sizeof(float) * ef.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(s->d_hist, 0, sizeof(double) * nc));
    HIP_TRY(hipMemset(s->d_hist_u, 0, sizeof(unsigned long long) * nc));
    *out = s.release();
    return DMC_OK;
}

dmc_status dmc_sample(dmc_sampler* s, uint64_t seed, uint64_t first_index, int64_t n, float* x, int64_t ld,
                      float* jac, void* stream) {
    if (!s || !x || !jac) return fail(DMC_E_INVALID, "null argument");
    if (n < 1 || ld < n) return fail(DMC_E_INVALID, "need n >= 1 and ld >= n");
    dmc::SampleArgs a;
    a.seed = seed;
    a.first = first_index;
    a.n = n;
    a.ld = ld;
    a.x = x;
    a.jac = jac;
    a.edges = s->d_edges;
    a.kind = s->kind;
    a.order = s->order;
    a.dim = s->dim;
    a.n_bins = s->n_bins;
    a.beta = (float)s->beta;
    a.qmax = (float)s->qmax;
    a.jl = (float)(4.0 * M_PI * s->qmax);
    a.jt = (float)std::pow(s->beta, s->order - 1);
    HIP_TRY(dmc::launch_sample(a, cu_count(), S(stream)));
    s->last_seed = seed;
    s->last_first = first_index;
    s->last_n = n;
    return DMC_OK;
}

dmc_status dmc_sampler_get_grid(const dmc_sampler* s, double* edges) {
    if (!s || !edges) return fail(DMC_E_INVALID, "null argument");
    std::copy(s->edges.begin(), s->edges.end(), edges);
    return DMC_OK;
}

dmc_status dmc_sampler_set_grid(dmc_sampler* s, const double* edges, void* stream) {
    if (!s || !edges) return fail(DMC_E_INVALID, "null argument");
    const int B = s->n_bins;
    for (int d = 0; d < s->dim; ++d) {
        const double* e = edges + (size_t)d * (B + 1);
        if (e[0] != 0.0 || e[B] != 1.0) return fail(DMC_E_INVALID, "grid must start at 0 and end at 1");
        for (int b = 0; b < B; ++b)
            if (!(e[b + 1] > e[b])) return fail(DMC_E_INVALID, "grid edges must rise strictly");
    }
    s->edges.assign(edges, edges + s->edges.size());
    std::vector<float> ef(s->edges.begin(), s->edges.end());
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipMemcpy(s->d_edges, ef.data(), sizeof(float) * ef.size(), hipMemcpyHostToDevice));
    return DMC_OK;
}

dmc_status dmc_sampler_read_histogram(dmc_sampler* s, double* hist, void* stream) {
    if (!s || !hist) return fail(DMC_E_INVALID, "null argument");
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipMemcpy(hist, s->d_hist, sizeof(double) * s->dim * s->n_bins, hipMemcpyDeviceToHost));
    return DMC_OK;
}

// VEGAS refinement (Lepage 1978), FP64 on the host: smooth each dimension's histogram with its
// neighbours, normalise, compress r -> ((1 - r) / ln(1/r))^alpha, then place the new edges so
// that every new bin holds an equal share of the compressed weight (uniform within old bins).
static void refine_dim(const double* e, const double* h, int B, double alpha, double* out) {
    std::vector<double> sm(B), w(B);
    sm[0] = (h[0] + h[1]) / 2;
    sm[B - 1] = (h[B - 2] + h[B - 1]) / 2;
    for (int b = 1; b < B - 1; ++b) sm[b] = (h[b - 1] + h[b] + h[b + 1]) / 3;
    double tot = 0;
    for (double v : sm) tot += v;
    if (!(tot > 0) || !std::isfinite(tot)) {
        std::copy(e, e + B + 1, out);
        return;
    }
    double wsum = 0;
    for (int b = 0; b < B; ++b) {
        const double r = sm[b] / tot;
        w[b] = r >= 1.0 ? 1.0 : (r > 0 ? std::pow((1.0 - r) / std::log(1.0 / r), alpha) : 0.0);
        wsum += w[b];
    }
    const double per = wsum / B;
    out[0] = 0.0;
    out[B] = 1.0;
    double acc = 0;
    int ob = 0;
    for (int j = 1; j < B; ++j) {
        const double target = j * per;
        while (ob < B && acc + w[ob] < target) acc += w[ob++];
        out[j] = e[ob] + (target - acc) / w[ob] * (e[ob + 1] - e[ob]);
    }
}

dmc_status dmc_vegas_refine(int32_t dim, int32_t n_bins, const double* edges, const double* hist, double alpha,
                            double* out) {
    if (!edges || !hist || !out) return fail(DMC_E_INVALID, "null argument");
    if (dim < 1 || n_bins < 2) return fail(DMC_E_INVALID, "need dim >= 1 and n_bins >= 2");
    if (!(alpha >= 0)) return fail(DMC_E_INVALID, "alpha must be >= 0");
    const int B = n_bins;
    for (int d = 0; d < dim; ++d)
        refine_dim(&edges[(size_t)d * (B + 1)], &hist[(size_t)d * B], B, alpha, &out[(size_t)d * (B + 1)]);
    // keep strictly rising edges (guard against empty histogram cells rounding to equal edges)
    for (int d = 0; d < dim; ++d)
        for (int b = 0; b < B; ++b) {
            const double lo = out[(size_t)d * (B + 1) + b];
            const double hi = out[(size_t)d * (B + 1) + b + 1];
            if (!(hi > lo)) {
                std::copy(&edges[(size_t)d * (B + 1)], &edges[(size_t)d * (B + 1)] + B + 1, &out[(size_t)d * (B + 1)]);
                break;
            }
        }
    return DMC_OK;
}

dmc_status dmc_sampler_refine(dmc_sampler* s, double alpha, void* stream) {
    if (!s) return fail(DMC_E_INVALID, "null sampler");
    if (s->kind != DMC_SAMPLER_VEGAS) return fail(DMC_E_STATE, "only a VEGAS sampler has a grid");
    if (!(alpha >= 0)) return fail(DMC_E_INVALID, "alpha must be >= 0");
    const int B = s->n_bins;
    std::vector<double> h((size_t)s->dim * B);
    dmc_status st = dmc_sampler_read_histogram(s, h.data(), stream);
    if (st != DMC_OK) return st;
    std::vector<double> ne(s->edges.size());
    st = dmc_vegas_refine(s->dim, B, s->edges.data(), h.data(), alpha, ne.data());
    if (st != DMC_OK) return st;
    s->edges = ne;
    std::vector<float> ef(ne.begin(), ne.end());
    HIP_TRY(hipMemcpy(s->d_edges, ef.data(), sizeof(float) * ef.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(s->d_hist, 0, sizeof(double) * s->dim * B));
    return DMC_OK;
}

void dmc_sampler_destroy(dmc_sampler* s) {
    if (!s) return;
    (void)hipFree(s->d_edges);
    (void)hipFree(s->d_hist);
    (void)hipFree(s->d_hist_u);
    (void)hipFree(s->d_max);
    delete s;
}

}  // extern "C"

// ------------------------------------------------------------------------------ flow
struct dmc_flow {
    int dim = 0, n_layers = 0;
    std::vector<int8_t> masks;
    int* d_aidx = nullptr;
    int* d_bidx = nullptr;
    int* d_dA = nullptr;
    float* master = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    __bf16* shadow = nullptr;
    int64_t step = 0;
    // training scratch
    int64_t cap_n = 0;
    int cap_part = 0;
    float* states = nullptr;
    float* G = nullptr;
    float* weff = nullptr;
    float* loss_part = nullptr;
    __bf16* acts = nullptr;
    float* partial = nullptr;
    double* sums = nullptr;
    float* mix_buf = nullptr;  // mixture scratch: log q, J_V, u' of the uniform share
    float* walk_buf = nullptr;  // base points of a random walk, [D][walk_cap]
    int64_t walk_cap = 0;
    int64_t mix_cap = 0;
    // kind 1: rational-quadratic spline couplings (FP32 parameters in `master`, no shadow)
    int kind = 0;
    int64_t n_params = 0;
    std::vector<int> offs_h, dA_h, aidx_h, bidx_h;  // [L], [L], [L][NSF_MAXD], [L][NSF_MAXD]
    int* d_offs = nullptr;
    float* s_grad = nullptr;   // [n_params]
    float* s_zs = nullptr;     // [L + 1][D][cap]
    float* s_adj = nullptr;    // [D][cap]
    float* s_vec = nullptr;    // per-sample vectors of one layer's reverse step
    float* s_partial = nullptr;
    float* s_lq = nullptr;     // [cap]
    int64_t s_cap = 0;
};

namespace {
void free_spline_train(dmc_flow* f) {
    (void)hipFree(f->s_zs);
    (void)hipFree(f->s_adj);
    (void)hipFree(f->s_vec);
    (void)hipFree(f->s_partial);
    (void)hipFree(f->s_lq);
    f->s_zs = f->s_adj = f->s_vec = f->s_partial = f->s_lq = nullptr;
    f->s_cap = 0;
}

void free_train(dmc_flow* f) {
    (void)hipFree(f->states);
    (void)hipFree(f->G);
    (void)hipFree(f->weff);
    (void)hipFree(f->loss_part);
    (void)hipFree(f->acts);
    (void)hipFree(f->partial);
    f->states = f->G = f->weff = f->loss_part = f->partial = nullptr;
    f->acts = nullptr;
    f->cap_n = 0;
    f->cap_part = 0;
}
constexpr int kActRows = dmc::FKIN + dmc::FH + dmc::FH + dmc::FNOUT + dmc::FH + dmc::FH;  // 560
constexpr int kWgradChunk = 1024;
}  // namespace

static void train_args(dmc_flow* f, dmc::FlowTrainArgs& a, int64_t n);
static dmc::NsfArgs nsf_args(dmc_flow* f, dmc_sampler* s);

extern "C" {

dmc_status dmc_flow_create(int32_t dim, int32_t n_layers, const int8_t* masks, dmc_flow** out) {
    if (!masks || !out) return fail(DMC_E_INVALID, "null argument");
    if (dim != 3 && dim != 7 && dim != 11 && dim != 15 && dim != 19 && dim != 23)
        return fail(DMC_E_INVALID, "dim must be 4n - 1 for an order n in 1..6");
    if (n_layers < 1 || n_layers > 32) return fail(DMC_E_INVALID, "n_layers in 1..32");
    std::vector<int> aidx(n_layers * 16, 0), bidx(n_layers * 16, 0), dA(n_layers);
    for (int l = 0; l < n_layers; ++l) {
        int na = 0, nb = 0;
        for (int d = 0; d < dim; ++d) {
            const int8_t mk = masks[l * dim + d];
            if (mk == 1) {
                if (na == 15) return fail(DMC_E_INVALID, "at most 15 conditioning dimensions per layer");
                aidx[l * 16 + na++] = d;
            } else if (mk == 0) {
                if (nb == 16) return fail(DMC_E_INVALID, "at most 16 transformed dimensions per layer");
                bidx[l * 16 + nb++] = d;
            } else {
                return fail(DMC_E_INVALID, "mask entries must be 0 or 1");
            }
        }
        if (na == 0 || nb == 0) return fail(DMC_E_INVALID, "every layer needs both parts");
        dA[l] = na;
    }
    auto f = std::make_unique<dmc_flow>();
    f->dim = dim;
    f->n_layers = n_layers;
    f->masks.assign(masks, masks + (size_t)n_layers * dim);
    const size_t P = (size_t)n_layers * dmc::LAYER_SIZE;
    HIP_ALLOC(hipMalloc(&f->d_aidx, sizeof(int) * aidx.size()));
    HIP_ALLOC(hipMalloc(&f->d_bidx, sizeof(int) * bidx.size()));
    HIP_ALLOC(hipMalloc(&f->d_dA, sizeof(int) * dA.size()));
    HIP_ALLOC(hipMalloc(&f->master, sizeof(float) * P));
    HIP_ALLOC(hipMalloc(&f->m, sizeof(float) * P));
    HIP_ALLOC(hipMalloc(&f->v, sizeof(float) * P));
    HIP_ALLOC(hipMalloc(&f->shadow, sizeof(__bf16) * (size_t)n_layers * dmc::SHADOW_LAYER));
    HIP_ALLOC(hipMalloc(&f->sums, sizeof(double) * 4));
    HIP_TRY(hipMemcpy(f->d_aidx, aidx.data(), sizeof(int) * aidx.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_bidx, bidx.data(), sizeof(int) * bidx.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_dA, dA.data(), sizeof(int) * dA.size(), hipMemcpyHostToDevice));
    // identity flow until parameters are set: all zero (the shadow's padding rows stay zero)
    HIP_TRY(hipMemset(f->master, 0, sizeof(float) * P));
    HIP_TRY(hipMemset(f->m, 0, sizeof(float) * P));
    HIP_TRY(hipMemset(f->v, 0, sizeof(float) * P));
    HIP_TRY(hipMemset(f->shadow, 0, sizeof(__bf16) * (size_t)n_layers * dmc::SHADOW_LAYER));
    *out = f.release();
    return DMC_OK;
}

dmc_status dmc_flow_create_spline(int32_t dim, int32_t n_layers, const int8_t* masks, dmc_flow** out) {
    if (!masks || !out) return fail(DMC_E_INVALID, "null argument");
    if (dim != 3 && dim != 7 && dim != 11 && dim != 15 && dim != 19 && dim != 23)
        return fail(DMC_E_INVALID, "dim must be 4n - 1 for an order n in 1..6");
    if (n_layers < 1 || n_layers > 32) return fail(DMC_E_INVALID, "n_layers in 1..32");
    const int MD = dmc::NSF_MAXD, H = dmc::NSF_H;
    auto f = std::make_unique<dmc_flow>();
    f->kind = 1;
    f->dim = dim;
    f->n_layers = n_layers;
    f->masks.assign(masks, masks + (size_t)n_layers * dim);
    f->aidx_h.assign((size_t)n_layers * MD, 0);
    f->bidx_h.assign((size_t)n_layers * MD, 0);
    f->dA_h.assign(n_layers, 0);
    f->offs_h.assign(n_layers, 0);
    int64_t off = 0;
    for (int l = 0; l < n_layers; ++l) {
        int na = 0, nb = 0;
        for (int d = 0; d < dim; ++d) {
            const int8_t mk = masks[l * dim + d];
            if (mk == 1)
                f->aidx_h[l * MD + na++] = d;
            else if (mk == 0)
                f->bidx_h[l * MD + nb++] = d;
            else
                return fail(DMC_E_INVALID, "mask entries must be 0 or 1");
        }
        if (na == 0 || nb == 0) return fail(DMC_E_INVALID, "every layer needs both parts");
        f->dA_h[l] = na;
        f->offs_h[l] = (int)off;
        const int P = dmc::NSF_NP * nb;
        const int count = H * na + H + H * H + H + P * H + P;
        off += count;
    }
    f->n_params = off;
    HIP_ALLOC(hipMalloc(&f->d_aidx, sizeof(int) * f->aidx_h.size()));
    HIP_ALLOC(hipMalloc(&f->d_bidx, sizeof(int) * f->bidx_h.size()));
    HIP_ALLOC(hipMalloc(&f->d_dA, sizeof(int) * n_layers));
    HIP_ALLOC(hipMalloc(&f->d_offs, sizeof(int) * n_layers));
    HIP_ALLOC(hipMalloc(&f->master, sizeof(float) * (size_t)off));
    HIP_ALLOC(hipMalloc(&f->m, sizeof(float) * (size_t)off));
    HIP_ALLOC(hipMalloc(&f->v, sizeof(float) * (size_t)off));
    HIP_ALLOC(hipMalloc(&f->s_grad, sizeof(float) * (size_t)off));
    HIP_ALLOC(hipMalloc(&f->sums, sizeof(double) * 4));
    HIP_TRY(hipMemcpy(f->d_aidx, f->aidx_h.data(), sizeof(int) * f->aidx_h.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_bidx, f->bidx_h.data(), sizeof(int) * f->bidx_h.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_dA, f->dA_h.data(), sizeof(int) * n_layers, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_offs, f->offs_h.data(), sizeof(int) * n_layers, hipMemcpyHostToDevice));
    // the identity flow until parameters are set: the output layer zero, interior-derivative biases at
    // softplus^-1(1 - 1e-3) (all spline derivatives 1, widths and heights equal), and He-normal hidden
    // weights from a fixed seed (zero hidden weights would leave every conditioner gradient but the
    // output biases' zero)
    std::vector<float> init((size_t)off, 0.0f);
    const float dzero = (float)std::log(std::exp(1.0 - 1e-3) - 1.0);
    uint64_t st = 0x5EEDF10Full;
    auto normal = [&st]() {  // splitmix64 uniforms, Box-Muller
        auto next = [&st]() {
            uint64_t z = (st += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return ((double)((z ^ (z >> 31)) >> 11) + 0.5) * 0x1p-53;
        };
        const double u1 = next(), u2 = next();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (int l = 0; l < n_layers; ++l) {
        const int na = f->dA_h[l], nb = dim - na, P = dmc::NSF_NP * nb;
        const size_t o = (size_t)f->offs_h[l];
        for (int i = 0; i < H * na; ++i) init[o + i] = (float)(normal() * std::sqrt(2.0 / na));
        for (int i = 0; i < H * H; ++i) init[o + H * na + H + i] = (float)(normal() * std::sqrt(2.0 / H));
        const size_t b3 = o + H * na + H + H * H + H + (size_t)P * H;
        for (int j = 0; j < nb; ++j)
            for (int r = 2 * dmc::NSF_K; r < dmc::NSF_NP; ++r) init[b3 + j * dmc::NSF_NP + r] = dzero;
    }
    HIP_TRY(hipMemcpy(f->master, init.data(), sizeof(float) * init.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(f->m, 0, sizeof(float) * (size_t)off));
    HIP_TRY(hipMemset(f->v, 0, sizeof(float) * (size_t)off));
    *out = f.release();
    return DMC_OK;
}

dmc_status dmc_flow_param_count(const dmc_flow* f, int64_t* n) {
    if (!f || !n) return fail(DMC_E_INVALID, "null argument");
    *n = f->kind == 1 ? f->n_params : (int64_t)f->n_layers * dmc::LAYER_SIZE;
    return DMC_OK;
}

dmc_status dmc_flow_set_params(dmc_flow* f, const float* theta, void* stream) {
    if (!f || !theta) return fail(DMC_E_INVALID, "null argument");
    const size_t P = f->kind == 1 ? (size_t)f->n_params : (size_t)f->n_layers * dmc::LAYER_SIZE;
    for (size_t i = 0; i < P; ++i)
        if (!std::isfinite(theta[i])) return fail(DMC_E_INVALID, "parameters must be finite");
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipMemcpy(f->master, theta, sizeof(float) * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(f->m, 0, sizeof(float) * P));
    HIP_TRY(hipMemset(f->v, 0, sizeof(float) * P));
    f->step = 0;
    if (f->kind == 0) HIP_TRY(dmc::launch_flow_shadow(f->master, f->shadow, f->n_layers, cu_count(), S(stream)));
    return DMC_OK;
}

dmc_status dmc_flow_get_params(dmc_flow* f, float* theta, void* stream) {
    if (!f || !theta) return fail(DMC_E_INVALID, "null argument");
    HIP_TRY(hipStreamSynchronize(S(stream)));
    const size_t P = f->kind == 1 ? (size_t)f->n_params : (size_t)f->n_layers * dmc::LAYER_SIZE;
    HIP_TRY(hipMemcpy(theta, f->master, sizeof(float) * P, hipMemcpyDeviceToHost));
    return DMC_OK;
}

dmc_status dmc_flow_sample(dmc_flow* f, dmc_sampler* s, uint64_t seed, uint64_t first, int64_t n, float* x,
                           int64_t ld, float* jac, float* u_out, float* lq_out, double mix_flow, double mix_uniform,
                           void* stream) {
    if (!f || !s || !x || !jac) return fail(DMC_E_INVALID, "null argument");
    if (s->dim != f->dim || s->kind != DMC_SAMPLER_VEGAS) return fail(DMC_E_INVALID, "need a VEGAS sampler of the flow's dimension");
    if (n < 1 || ld < n) return fail(DMC_E_INVALID, "need n >= 1 and ld >= n");
    if (!(mix_flow > 0.0 && mix_flow <= 1.0) || !(mix_uniform >= 0.0 && mix_uniform < 1.0) ||
        mix_flow + mix_uniform > 1.0 + 1e-12)
        return fail(DMC_E_INVALID, "mixture shares: flow in (0, 1], uniform in [0, 1), flow + uniform <= 1");
    const double mix_grid = std::max(0.0, 1.0 - mix_flow - mix_uniform);
    // balance-heuristic mixture: samples [0, n_u) uniform, [n_u, n_u + n_g) from the grid, the rest through the flow
    const int64_t n_u = std::min<int64_t>(n, (int64_t)std::llround(mix_uniform * (double)n));
    const int64_t n_g = std::min<int64_t>(n - n_u, (int64_t)std::llround(mix_grid * (double)n));
    const int64_t n_f = n - n_u - n_g;
    const int D = f->dim;
    const float af = (float)mix_flow, ag = (float)mix_grid, au = (float)mix_uniform;
    // scratch: log q and J_V of the uniform and grid shares, u' of the uniform share if u_out is NULL
    const int64_t need = 2 * (n_u + n_g) + (u_out ? 0 : (int64_t)D * n_u);
    if (need > 0 && f->mix_cap < need) {
        (void)hipFree(f->mix_buf);
        f->mix_buf = nullptr;
        f->mix_cap = 0;
        HIP_ALLOC(hipMalloc(&f->mix_buf, sizeof(float) * (size_t)need));
        f->mix_cap = need;
    }
    float* lq_s = f->mix_buf;
    float* jv_s = lq_s + (n_u + n_g);
    float* up_s = jv_s + (n_u + n_g);
    const int ncu = cu_count();
    if (n_u > 0) {
        dmc::FlowUniformArgs ua;
        ua.seed = seed;
        ua.first = first;
        ua.n = n_u;
        ua.ld = ld;
        ua.ldu = u_out ? ld : n_u;
        ua.x = x;
        ua.jac = jac;
        ua.u_out = u_out ? u_out : up_s;
        ua.jv_out = jv_s;
        ua.edges = s->d_edges;
        ua.n_bins = s->n_bins;
        ua.dim = D;
        ua.beta = (float)s->beta;
        ua.qmax = (float)s->qmax;
        ua.jl = (float)(4.0 * M_PI * s->qmax);
        ua.jt = (float)std::pow(s->beta, s->order - 1);
        HIP_TRY(dmc::launch_flow_uniform(ua, ncu, S(stream)));
        if (f->kind == 1) {
            dmc::NsfArgs na = nsf_args(f, s);
            na.u_in = u_out ? u_out : up_s;
            na.ld = u_out ? ld : n_u;
            na.n = n_u;
            na.lq_out = lq_out ? lq_out : lq_s;
            HIP_TRY(dmc::launch_nsf_inverse(na, ncu, S(stream)));
            HIP_TRY(dmc::launch_flow_mix(jac, na.lq_out, jv_s, n_u, af, ag, au, true, S(stream)));
        } else {
            dmc::FlowTrainArgs a;
            train_args(f, a, n_u);
            a.u_in = u_out ? u_out : up_s;
            a.ld = u_out ? ld : n_u;
            a.states = nullptr;
            a.G = nullptr;
            a.weff = nullptr;
            a.w = nullptr;
            a.loss_part = nullptr;
            a.lq_out = lq_out ? lq_out : lq_s;
            HIP_TRY(dmc::launch_flow_inverse(a, dmc::flow_inverse_blocks(n_u, ncu), S(stream)));
            HIP_TRY(dmc::launch_flow_mix(jac, a.lq_out, jv_s, n_u, af, ag, au, true, S(stream)));
        }
    }
    if (n_g > 0) {
        dmc_status st = dmc_sample(s, seed, first + (uint64_t)n_u, n_g, x + n_u, ld, jac + n_u, stream);
        if (st != DMC_OK) return st;
        if (f->kind == 1) {
            dmc::NsfArgs na = nsf_args(f, s);
            na.u_in = nullptr;
            na.seed = seed;
            na.first = first + (uint64_t)n_u;
            na.n = n_g;
            na.ld = ld;
            na.lq_out = lq_out ? lq_out + n_u : lq_s + n_u;
            na.u_out = u_out ? u_out + n_u : nullptr;
            na.jv_out = jv_s + n_u;
            HIP_TRY(dmc::launch_nsf_inverse(na, ncu, S(stream)));
            HIP_TRY(dmc::launch_flow_mix(jac + n_u, na.lq_out, jv_s + n_u, n_g, af, ag, au, false, S(stream)));
        } else {
            dmc::FlowTrainArgs a;
            train_args(f, a, n_g);
            a.u_in = nullptr;
            a.seed = seed;
            a.first = first + (uint64_t)n_u;
            a.ld = ld;
            a.states = nullptr;
            a.G = nullptr;
            a.weff = nullptr;
            a.w = nullptr;
            a.loss_part = nullptr;
            a.lq_out = lq_out ? lq_out + n_u : lq_s + n_u;
            a.u_out = u_out ? u_out + n_u : nullptr;
            a.edges = s->d_edges;
            a.n_bins = s->n_bins;
            a.jv_out = jv_s + n_u;
            HIP_TRY(dmc::launch_flow_inverse(a, dmc::flow_inverse_blocks(n_g, ncu), S(stream)));
            HIP_TRY(dmc::launch_flow_mix(jac + n_u, a.lq_out, jv_s + n_u, n_g, af, ag, au, false, S(stream)));
        }
    }
    if (n_f > 0 && f->kind == 1) {
        const int64_t o = n_u + n_g;
        dmc::NsfArgs na = nsf_args(f, s);
        na.seed = seed;
        na.first = first + (uint64_t)o;
        na.n = n_f;
        na.ld = ld;
        na.x = x + o;
        na.jac = jac + o;
        na.u_out = u_out ? u_out + o : nullptr;
        na.lq_out = lq_out ? lq_out + o : nullptr;
        na.mix_f = af;
        na.mix_g = ag;
        na.mix_u = au;
        HIP_TRY(dmc::launch_nsf_sample(na, ncu, S(stream)));
    } else if (n_f > 0) {
        const int64_t o = n_u + n_g;
        dmc::FlowSampleArgs a;
        a.seed = seed;
        a.first = first + (uint64_t)o;
        a.n = n_f;
        a.ld = ld;
        a.x = x + o;
        a.jac = jac + o;
        a.u_out = u_out ? u_out + o : nullptr;
        a.lq_out = lq_out ? lq_out + o : nullptr;
        a.edges = s->d_edges;
        a.master = f->master;
        a.shadow = f->shadow;
        a.aidx = f->d_aidx;
        a.bidx = f->d_bidx;
        a.dA = f->d_dA;
        a.n_layers = f->n_layers;
        a.n_bins = s->n_bins;
        a.beta = (float)s->beta;
        a.qmax = (float)s->qmax;
        a.jl = (float)(4.0 * M_PI * s->qmax);
        a.jt = (float)std::pow(s->beta, s->order - 1);
        a.mix_f = af;
        a.mix_g = ag;
        a.mix_u = au;
        HIP_TRY(dmc::launch_flow_sample(a, D, ncu, S(stream)));
    }
    s->last_n = -1;  // the grid histogram does not apply to mixture samples
    return DMC_OK;
}

// activation rows hold whole 16-sample slices (two aligned 16-byte loads per MFMA operand)
static int64_t act_stride(int64_t n) { return (n + 15) & ~(int64_t)15; }

static dmc_status flow_scratch(dmc_flow* f, int64_t n, int nblk) {
    if (n <= f->cap_n && nblk <= f->cap_part) return DMC_OK;
    free_train(f);
    const int64_t cn = std::max<int64_t>(n, 1024);
    const int cp = std::max(nblk, (int)((cn + kWgradChunk - 1) / kWgradChunk));
    HIP_ALLOC(hipMalloc(&f->states, sizeof(float) * (size_t)f->n_layers * f->dim * cn));
    HIP_ALLOC(hipMalloc(&f->G, sizeof(float) * (size_t)f->dim * cn));
    HIP_ALLOC(hipMalloc(&f->weff, sizeof(float) * (size_t)cn));
    HIP_ALLOC(hipMalloc(&f->acts, sizeof(__bf16) * (size_t)kActRows * act_stride(cn)));
    HIP_ALLOC(hipMalloc(&f->loss_part, sizeof(float) * (size_t)cp));
    HIP_ALLOC(hipMalloc(&f->partial, sizeof(float) * (size_t)f->n_layers * cp * dmc::LAYER_SIZE));
    f->cap_n = cn;
    f->cap_part = cp;
    return DMC_OK;
}

static void train_args(dmc_flow* f, dmc::FlowTrainArgs& a, int64_t n) {
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.master = f->master;
    a.shadow = f->shadow;
    a.aidx = f->d_aidx;
    a.bidx = f->d_bidx;
    a.dA = f->d_dA;
    a.n_layers = f->n_layers;
    a.dim = f->dim;
    a.states = f->states;
    a.G = f->G;
    a.weff = f->weff;
    a.loss_part = f->loss_part;
    a.lda = act_stride(n);
    if (!f->acts) return;  // density-only passes before any training scratch exists
    __bf16* p = f->acts;
    a.act_x1 = p;
    p += (size_t)dmc::FKIN * a.lda;
    a.act_h1 = p;
    p += (size_t)dmc::FH * a.lda;
    a.act_h2 = p;
    p += (size_t)dmc::FH * a.lda;
    a.act_do = p;
    p += (size_t)dmc::FNOUT * a.lda;
    a.act_dp2 = p;
    p += (size_t)dmc::FH * a.lda;
    a.act_dp1 = p;
}

static dmc::NsfArgs nsf_args(dmc_flow* f, dmc_sampler* s) {
    dmc::NsfArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = f->master;
    a.offs = f->d_offs;
    a.aidx = f->d_aidx;
    a.bidx = f->d_bidx;
    a.dA = f->d_dA;
    a.n_layers = f->n_layers;
    a.dim = f->dim;
    if (s) {
        a.edges = s->d_edges;
        a.n_bins = s->n_bins;
        a.beta = (float)s->beta;
        a.qmax = (float)s->qmax;
        a.jl = (float)(4.0 * M_PI * s->qmax);
        a.jt = (float)std::pow(s->beta, s->order - 1);
    }
    return a;
}

// One weighted forward-KL step of a spline flow: the inverse pass keeps every layer's points, then the
// layers' reverse steps run in application order (the adjoint of the base point is zero under the
// uniform base), each followed by its weight-gradient sums; finally Adam.
static dmc_status spline_train_step(dmc_flow* f, const float* u, int64_t ld, uint64_t seed, uint64_t first, int64_t n,
                                    const float* w, double lr, float* grad_out, double* loss, void* stream) {
    const int D = f->dim, L = f->n_layers, H = dmc::NSF_H;
    int maxP = 0, maxA = 0;
    for (int l = 0; l < L; ++l) {
        maxP = std::max(maxP, dmc::NSF_NP * (D - f->dA_h[l]));
        maxA = std::max(maxA, f->dA_h[l]);
    }
    if (n > f->s_cap) {
        free_spline_train(f);
        HIP_ALLOC(hipMalloc(&f->s_zs, sizeof(float) * (size_t)(L + 1) * D * n));
        HIP_ALLOC(hipMalloc(&f->s_adj, sizeof(float) * (size_t)D * n));
        HIP_ALLOC(hipMalloc(&f->s_vec, sizeof(float) * (size_t)(maxP + 4 * H + maxA) * n));
        HIP_ALLOC(hipMalloc(&f->s_partial, sizeof(float) * (size_t)dmc::nsf_outer_chunks(n) * maxP * (H + 1)));
        HIP_ALLOC(hipMalloc(&f->s_lq, sizeof(float) * (size_t)n));
        f->s_cap = n;
    }
    const int ncu = cu_count();
    dmc::NsfArgs na = nsf_args(f, nullptr);
    na.u_in = u;
    na.ld = u ? ld : n;
    na.seed = seed;
    na.first = first;
    na.n = n;
    na.lq_out = f->s_lq;
    na.zs = f->s_zs;
    HIP_TRY(dmc::launch_nsf_inverse(na, ncu, S(stream)));
    HIP_TRY(dmc::launch_nsf_loss(w, f->s_lq, n, f->sums, 1, S(stream)));
    HIP_TRY(hipMemsetAsync(f->s_adj, 0, sizeof(float) * (size_t)D * n, S(stream)));
    for (int l = 0; l < L; ++l) {
        const int dA = f->dA_h[l], dB = D - dA, P = dmc::NSF_NP * dB;
        dmc::NsfBackArgs b;
        b.params = f->master;
        b.off = f->offs_h[l];
        b.dA = dA;
        b.dB = dB;
        b.dim = D;
        b.aidx = f->d_aidx + l * dmc::NSF_MAXD;
        b.bidx = f->d_bidx + l * dmc::NSF_MAXD;
        b.z = f->s_zs + (size_t)(l + 1) * D * n;
        b.adj = f->s_adj;
        b.w = w;
        b.inv_wsum = f->sums + 2;
        b.n = n;
        float* v = f->s_vec;
        b.d_theta = v;
        v += (size_t)P * n;
        b.a2 = v;
        v += (size_t)H * n;
        b.d_pre2 = v;
        v += (size_t)H * n;
        b.a1 = v;
        v += (size_t)H * n;
        b.d_pre1 = v;
        v += (size_t)H * n;
        b.zA = v;
        HIP_TRY(dmc::launch_nsf_backward(b, ncu, S(stream)));
        float* g = f->s_grad + f->offs_h[l];
        // W1 [H][dA], b1 [H]; W2 [H][H], b2 [H]; W3 [P][H], b3 [P]
        HIP_TRY(dmc::launch_nsf_outer(b.d_pre1, H, b.zA, dA, n, f->s_partial, S(stream)));
        HIP_TRY(dmc::launch_nsf_outer_fold(f->s_partial, H, dA, n, g, S(stream)));
        HIP_TRY(dmc::launch_nsf_outer(b.d_pre2, H, b.a1, H, n, f->s_partial, S(stream)));
        HIP_TRY(dmc::launch_nsf_outer_fold(f->s_partial, H, H, n, g + H * dA + H, S(stream)));
        HIP_TRY(dmc::launch_nsf_outer(b.d_theta, P, b.a2, H, n, f->s_partial, S(stream)));
        HIP_TRY(dmc::launch_nsf_outer_fold(f->s_partial, P, H, n, g + H * dA + H + H * H + H, S(stream)));
    }
    if (grad_out)
        HIP_TRY(hipMemcpyAsync(grad_out, f->s_grad, sizeof(float) * (size_t)f->n_params, hipMemcpyDeviceToDevice,
                               S(stream)));
    if (lr > 0) {
        ++f->step;
        HIP_TRY(dmc::launch_nsf_adam(f->master, f->m, f->v, f->s_grad, f->n_params, f->step, (float)lr, S(stream)));
    }
    if (loss) {
        double h[4];
        HIP_TRY(hipStreamSynchronize(S(stream)));
        HIP_TRY(hipMemcpy(h, f->sums, sizeof(h), hipMemcpyDeviceToHost));
        *loss = h[3];
        if (!std::isfinite(h[0]) || !(h[0] > 0)) return fail(DMC_E_NUMERIC, "weights sum to zero or are not finite");
    }
    return DMC_OK;
}

dmc_status dmc_flow_walk(dmc_flow* f, dmc_sampler* s, const float* u_state, int64_t ld_u, int64_t n, double sigma,
                         uint64_t seed, uint64_t first, float* x, int64_t ld, float* jac, float* jac_flow, float* u_out,
                         float* jac_flow_state, double mix_flow, double mix_uniform, void* stream) {
    if (!f || !s || !u_state || !x || !jac || !jac_flow || !u_out || !jac_flow_state)
        return fail(DMC_E_INVALID, "null argument");
    if (f->kind != 1) return fail(DMC_E_INVALID, "the base-space walk is built for spline flows");
    if (s->dim != f->dim || s->kind != DMC_SAMPLER_VEGAS) return fail(DMC_E_INVALID, "need a VEGAS sampler of the flow's dimension");
    if (n < 1 || ld < n || ld_u < n) return fail(DMC_E_INVALID, "need n >= 1, ld >= n and ld_u >= n");
    if (!(sigma > 0.0 && sigma < 1e6)) return fail(DMC_E_INVALID, "sigma must be positive and finite");
    if (!(mix_flow > 0.0 && mix_flow <= 1.0) || !(mix_uniform >= 0.0 && mix_uniform < 1.0) ||
        mix_flow + mix_uniform > 1.0 + 1e-12)
        return fail(DMC_E_INVALID, "mixture shares: flow in (0, 1], uniform in [0, 1), flow + uniform <= 1");
    const int D = f->dim;
    if (f->walk_cap < n) {
        (void)hipFree(f->walk_buf);
        f->walk_buf = nullptr;
        f->walk_cap = 0;
        HIP_ALLOC(hipMalloc(&f->walk_buf, sizeof(float) * (size_t)D * (size_t)n));
        f->walk_cap = n;
    }
    const int ncu = cu_count();
    // the states' base points z = T^-1(u') and the flow's own weights there
    dmc::NsfArgs na = nsf_args(f, s);
    na.u_in = u_state;
    na.ld = ld_u;
    na.n = n;
    na.z0_out = f->walk_buf;
    na.ld_z = n;
    na.jf_out = jac_flow_state;
    HIP_TRY(dmc::launch_nsf_inverse(na, ncu, S(stream)));
    // the symmetric move, then the flow from the moved base points: proposals with their mixture weight
    // (for the target) and the flow's own weight (for the test)
    HIP_TRY(dmc::launch_nsf_walk(f->walk_buf, D, n, n, (float)sigma, seed, first, ncu, S(stream)));
    dmc::NsfArgs sa = nsf_args(f, s);
    sa.z_in = f->walk_buf;
    sa.ld_z = n;
    sa.n = n;
    sa.ld = ld;
    sa.x = x;
    sa.jac = jac;
    sa.jf_out = jac_flow;
    sa.u_out = u_out;
    sa.mix_f = (float)mix_flow;
    sa.mix_g = (float)std::max(0.0, 1.0 - mix_flow - mix_uniform);
    sa.mix_u = (float)mix_uniform;
    HIP_TRY(dmc::launch_nsf_sample(sa, ncu, S(stream)));
    return DMC_OK;
}

dmc_status dmc_flow_log_density(dmc_flow* f, const float* u, int64_t ld, int64_t n, float* lq, void* stream) {
    if (!f || !u || !lq) return fail(DMC_E_INVALID, "null argument");
    if (n < 1 || ld < n) return fail(DMC_E_INVALID, "need n >= 1 and ld >= n");
    if (f->kind == 1) {
        dmc::NsfArgs na = nsf_args(f, nullptr);
        na.u_in = u;
        na.ld = ld;
        na.n = n;
        na.lq_out = lq;
        HIP_TRY(dmc::launch_nsf_inverse(na, cu_count(), S(stream)));
        return DMC_OK;
    }
    const int nblk = dmc::flow_inverse_blocks(n, cu_count());
    dmc::FlowTrainArgs a;
    train_args(f, a, n);
    a.u_in = u;
    a.ld = ld;
    a.states = nullptr;
    a.G = nullptr;
    a.weff = nullptr;
    a.w = nullptr;
    a.loss_part = nullptr;
    a.lq_out = lq;
    HIP_TRY(dmc::launch_flow_inverse(a, nblk, S(stream)));
    return DMC_OK;
}

dmc_status dmc_flow_train_step(dmc_flow* f, const float* u, int64_t ld, uint64_t seed, uint64_t first, int64_t n,
                               const float* w, double lr, float* grad_out, double* loss, void* stream) {
    if (!f || !w) return fail(DMC_E_INVALID, "null argument");
    if (n < 1 || (u && ld < n)) return fail(DMC_E_INVALID, "need n >= 1 and ld >= n");
    if (!(lr >= 0)) return fail(DMC_E_INVALID, "lr must be >= 0");
    if (f->kind == 1) return spline_train_step(f, u, ld, seed, first, n, w, lr, grad_out, loss, stream);
    const int ncu = cu_count();
    const int nblk = dmc::flow_train_blocks(n, ncu);
    const int nblk_inv = dmc::flow_inverse_blocks(n, ncu);
    const int wg_blocks = (int)((n + kWgradChunk - 1) / kWgradChunk);
    dmc_status st = flow_scratch(f, n, std::max(std::max(nblk, nblk_inv), wg_blocks));
    if (st != DMC_OK) return st;
    dmc::FlowTrainArgs a;
    train_args(f, a, n);
    a.u_in = u;
    a.ld = u ? ld : n;
    a.seed = seed;
    a.first = first;
    a.w = w;
    a.inv_wsum = f->sums + 2;
    HIP_TRY(dmc::launch_flow_sums(w, n, f->sums, S(stream)));
    HIP_TRY(dmc::launch_flow_inverse(a, nblk_inv, S(stream)));
    for (int l = 0; l < f->n_layers; ++l)
        HIP_TRY(dmc::launch_flow_backward(a, nblk, l, kWgradChunk, wg_blocks,
                                          f->partial + (size_t)l * f->cap_part * dmc::LAYER_SIZE, S(stream)));
    HIP_TRY(dmc::launch_flow_loss(f->loss_part, nblk_inv, f->sums, S(stream)));
    dmc::FlowAdamArgs ad;
    ad.partial = f->partial;
    ad.nblk = wg_blocks;
    ad.nblk_max = f->cap_part;
    ad.n_layers = f->n_layers;
    ad.apply = lr > 0;
    ad.master = f->master;
    ad.m = f->m;
    ad.v = f->v;
    ad.shadow = f->shadow;
    ad.grad_out = grad_out;
    ad.lr = lr;
    ad.b1 = 0.9;
    ad.b2 = 0.999;
    ad.eps = 1e-8;
    if (lr > 0) ++f->step;
    ad.b1t = std::pow(ad.b1, (double)std::max<int64_t>(f->step, 1));
    ad.b2t = std::pow(ad.b2, (double)std::max<int64_t>(f->step, 1));
    HIP_TRY(dmc::launch_flow_adam(ad, ncu, S(stream)));
    if (loss) {
        double h[4];
        HIP_TRY(hipStreamSynchronize(S(stream)));
        HIP_TRY(hipMemcpy(h, f->sums, sizeof(h), hipMemcpyDeviceToHost));
        *loss = h[1];
        if (!std::isfinite(h[0]) || !(h[0] > 0)) return fail(DMC_E_NUMERIC, "weights sum to zero or are not finite");
    }
    return DMC_OK;
}

void dmc_flow_destroy(dmc_flow* f) {
    if (!f) return;
    free_train(f);
    free_spline_train(f);
    (void)hipFree(f->d_offs);
    (void)hipFree(f->s_grad);
    (void)hipFree(f->d_aidx);
    (void)hipFree(f->d_bidx);
    (void)hipFree(f->d_dA);
    (void)hipFree(f->master);
    (void)hipFree(f->m);
    (void)hipFree(f->v);
    (void)hipFree(f->shadow);
    (void)hipFree(f->sums);
    (void)hipFree(f->mix_buf);
    (void)hipFree(f->walk_buf);
    delete f;
}


// ------------------------------------------------------------------------------ Markov chains
}  // extern "C"

struct dmc_chains {
    int64_t n = 0;
    int n_batches = 0, n_groups = 0, n_k = 0, n_roots = 0, S = 0, D = 0;
    float* f_state = nullptr;     // device [S][n]
    float* u_state = nullptr;     // device [D][n] (D > 0)
    double* q_state = nullptr;    // device [n]
    double* pi_state = nullptr;   // device [n]
    double* partial = nullptr;    // device [nblk][n_batches][S + 1][2]: per-block running sums since the last fold
    double* totals = nullptr;     // device [n_batches][S + 1][2]
    unsigned int* zeros = nullptr;              // device [nblk] (the fold's count column, unused)
    unsigned long long* nonfin = nullptr;       // device, the fold's count (unused)
    unsigned long long* n_acc = nullptr;        // device: accepted proposals since the last reset
    int nblk = 0, chunk = 0;      // accumulate blocks per batch, chains per block
    int64_t steps = 0, measured = 0;
    bool unfolded = false;        // partial holds measured steps not yet in totals
    size_t totals_len() const { return (size_t)n_batches * (S + 1) * 2; }
};

extern "C" {

dmc_status dmc_chains_create(int64_t n, int32_t n_batches, int32_t n_groups, int32_t n_k, int32_t n_roots,
                             int32_t dim_u, dmc_chains** out) {
    if (!out || n < 1 || n_groups < 1 || n_groups > DMC_MAX_GROUPS || n_k < 1 || n_k > DMC_MAX_K || n_roots < 1 ||
        n_roots > DMC_MAX_ROOTS)
        return fail(DMC_E_INVALID, "chain count or observable shape out of range");
    if (n_batches < 1 || n_batches > DMC_MAX_CHAIN_BATCHES || n_batches > n)
        return fail(DMC_E_INVALID, "n_batches must be in [1, min(n, DMC_MAX_CHAIN_BATCHES)]");
    if (dim_u < 0 || dim_u > 4 * DMC_MAX_ORDER - 1) return fail(DMC_E_INVALID, "dim_u must be in 0..4 DMC_MAX_ORDER - 1");
    auto c = std::make_unique<dmc_chains>();
    c->n = n;
    c->n_batches = n_batches;
    c->n_groups = n_groups;
    c->n_k = n_k;
    c->n_roots = n_roots;
    c->S = n_groups * n_roots * n_k * 2;
    c->nblk = dmc::mcmc_acc_blocks((n + n_batches - 1) / n_batches, &c->chunk);
    HIP_ALLOC(hipMalloc(&c->f_state, sizeof(float) * (size_t)c->S * n));
    c->D = dim_u;
    if (dim_u > 0) HIP_ALLOC(hipMalloc(&c->u_state, sizeof(float) * (size_t)dim_u * n));
    HIP_ALLOC(hipMalloc(&c->q_state, sizeof(double) * (size_t)n));
    HIP_ALLOC(hipMalloc(&c->pi_state, sizeof(double) * (size_t)n));
    HIP_ALLOC(hipMalloc(&c->partial, sizeof(double) * (size_t)c->nblk * c->totals_len()));
    HIP_ALLOC(hipMalloc(&c->totals, sizeof(double) * c->totals_len()));
    HIP_ALLOC(hipMalloc(&c->zeros, sizeof(unsigned int) * (size_t)c->nblk));
    HIP_ALLOC(hipMalloc(&c->nonfin, sizeof(unsigned long long)));
    HIP_ALLOC(hipMalloc(&c->n_acc, sizeof(unsigned long long)));
    HIP_TRY(hipMemset(c->totals, 0, sizeof(double) * c->totals_len()));
    HIP_TRY(hipMemset(c->partial, 0, sizeof(double) * (size_t)c->nblk * c->totals_len()));
    HIP_TRY(hipMemset(c->zeros, 0, sizeof(unsigned int) * (size_t)c->nblk));
    HIP_TRY(hipMemset(c->nonfin, 0, sizeof(unsigned long long)));
    HIP_TRY(hipMemset(c->n_acc, 0, sizeof(unsigned long long)));
    *out = c.release();
    return DMC_OK;
}

static dmc_status chains_step(dmc_chains* c, const float* f_prop, int64_t ld, const float* jac_prop, const float* g_prop,
                              const float* g_state, const float* u_prop, int64_t ld_u, int64_t offset, double alpha,
                              uint64_t seed, int32_t measure, void* stream) {
    dmc::McmcArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g_prop = g_prop;
    a.g_state = g_state;
    a.n = c->n;
    a.S = c->S;
    a.R = c->n_roots;
    a.K = c->n_k;
    a.G = c->n_groups;
    a.f_prop = f_prop;
    a.ld_prop = ld;
    a.jac_prop = jac_prop;
    a.offset = offset;
    a.D = c->D;
    a.u_prop = u_prop;
    a.ld_u = ld_u;
    a.u_state = c->u_state;
    a.f_state = c->f_state;
    a.q_state = c->q_state;
    a.pi_state = c->pi_state;
    a.alpha = alpha;
    a.seed = seed;
    a.step = (uint64_t)c->steps;
    a.first = c->steps == 0;
    a.n_acc = c->n_acc;
    HIP_TRY(dmc::launch_mcmc_accept(a, cu_count(), S(stream)));
    ++c->steps;
    if (measure) {
        dmc::McmcAccArgs m;
        m.n = c->n;
        m.S = c->S;
        m.n_batches = c->n_batches;
        m.f_state = c->f_state;
        m.q_state = c->q_state;
        m.pi_state = c->pi_state;
        m.partial = c->partial;
        m.chunk = c->chunk;
        HIP_TRY(dmc::launch_mcmc_accumulate(m, c->nblk, S(stream)));
        c->unfolded = true;
        c->measured += c->n;
    }
    return DMC_OK;
}

dmc_status dmc_chains_step(dmc_chains* c, const float* f_prop, int64_t ld, const float* jac_prop, const float* u_prop,
                           int64_t ld_u, int64_t offset, double alpha, uint64_t seed, int32_t measure, void* stream) {
    if (!c || !f_prop || !jac_prop) return fail(DMC_E_INVALID, "null argument");
    if (ld < c->n) return fail(DMC_E_INVALID, "ld must be at least the chain count");
    if (c->D > 0 && (!u_prop || ld_u < c->n))
        return fail(DMC_E_INVALID, "chains that keep coordinates need u_prop with ld_u >= the chain count");
    if (offset < 0 || offset >= c->n) return fail(DMC_E_INVALID, "offset must be in [0, n)");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(DMC_E_INVALID, "alpha must be in [0, 1]");
    return chains_step(c, f_prop, ld, jac_prop, nullptr, nullptr, u_prop, ld_u, offset, alpha, seed, measure, stream);
}

dmc_status dmc_chains_step_walk(dmc_chains* c, const float* f_prop, int64_t ld, const float* jac_prop,
                                const float* jac_flow_prop, const float* jac_flow_state, const float* u_prop,
                                int64_t ld_u, double alpha, uint64_t seed, int32_t measure, void* stream) {
    if (!c || !f_prop || !jac_prop || !jac_flow_prop || !jac_flow_state || !u_prop)
        return fail(DMC_E_INVALID, "null argument");
    if (c->D == 0) return fail(DMC_E_INVALID, "a walk needs chains that keep their coordinates (dim_u > 0)");
    if (ld < c->n || ld_u < c->n) return fail(DMC_E_INVALID, "ld and ld_u must be at least the chain count");
    if (c->steps == 0) return fail(DMC_E_INVALID, "a walk moves existing states: take an independence step first");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(DMC_E_INVALID, "alpha must be in [0, 1]");
    return chains_step(c, f_prop, ld, jac_prop, jac_flow_prop, jac_flow_state, u_prop, ld_u, 0, alpha, seed, measure,
                       stream);
}

// the per-block running sums into the totals (fixed order), then cleared
static dmc_status chains_fold(dmc_chains* c, void* stream) {
    if (!c->unfolded) return DMC_OK;
    HIP_TRY(dmc::launch_fold(c->partial, c->nblk, (int)c->totals_len(), c->totals, c->zeros, c->nonfin, S(stream)));
    HIP_TRY(hipMemsetAsync(c->partial, 0, sizeof(double) * (size_t)c->nblk * c->totals_len(), S(stream)));
    c->unfolded = false;
    return DMC_OK;
}

dmc_status dmc_chains_read(dmc_chains* c, double* sums, int64_t* n_measured, int64_t* n_accepted, void* stream) {
    if (!c || !sums) return fail(DMC_E_INVALID, "null argument");
    unsigned long long acc = 0;
    dmc_status st = chains_fold(c, stream);
    if (st != DMC_OK) return st;
    HIP_TRY(hipStreamSynchronize(S(stream)));
    HIP_TRY(hipMemcpy(sums, c->totals, sizeof(double) * c->totals_len(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&acc, c->n_acc, sizeof(acc), hipMemcpyDeviceToHost));
    if (n_measured) *n_measured = c->measured;
    if (n_accepted) *n_accepted = (int64_t)acc;
    return DMC_OK;
}

dmc_status dmc_chains_training_data(dmc_chains* c, float* u, int64_t ld, float* w, void* stream) {
    if (!c || !w || (c->D > 0 && !u)) return fail(DMC_E_INVALID, "null argument");
    if (c->D > 0 && ld < c->n) return fail(DMC_E_INVALID, "ld must be at least the chain count");
    if (c->steps == 0) return fail(DMC_E_STATE, "the chains have no state yet");
    dmc::McmcTrainArgs a;
    a.n = c->n;
    a.S = c->S;
    a.R = c->n_roots;
    a.K = c->n_k;
    a.G = c->n_groups;
    a.D = c->D;
    a.f_state = c->f_state;
    a.pi_state = c->pi_state;
    a.u_state = c->u_state;
    a.u_out = u;
    a.ld_out = ld;
    a.w_out = w;
    HIP_TRY(dmc::launch_mcmc_training(a, cu_count(), S(stream)));
    return DMC_OK;
}

dmc_status dmc_chains_reset(dmc_chains* c, void* stream) {
    if (!c) return fail(DMC_E_INVALID, "null argument");
    HIP_TRY(hipMemsetAsync(c->totals, 0, sizeof(double) * c->totals_len(), S(stream)));
    HIP_TRY(hipMemsetAsync(c->partial, 0, sizeof(double) * (size_t)c->nblk * c->totals_len(), S(stream)));
    c->unfolded = false;
    HIP_TRY(hipMemsetAsync(c->n_acc, 0, sizeof(unsigned long long), S(stream)));
    c->measured = 0;
    return DMC_OK;
}

// the rotation offset of step t: splitmix64 (Steele, Lea and Flood 2014) of the key and step, reduced to [0, n)
static int64_t chain_offset(uint64_t key, uint64_t t, int64_t n) {
    uint64_t z = key + (t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (int64_t)(((unsigned __int128)z * (uint64_t)n) >> 64);
}

dmc_status dmc_chains_run(dmc_chains* c, dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext,
                          int32_t n_k, dmc_sampler* s, dmc_flow* flow, double mix_flow, double mix_uniform,
                          uint64_t seed, uint64_t first, int64_t thermal, int64_t steps, double alpha,
                          uint64_t accept_seed, uint64_t offset_key, float* x, int64_t ld, float* jac, float* f,
                          float* u, dmc_accum* acc, void* stream) {
    if (!c || !g || !inst || !k_ext || !s || !x || !jac || !f || !acc) return fail(DMC_E_INVALID, "null argument");
    if (thermal < 0 || steps < 0) return fail(DMC_E_INVALID, "thermal and steps must be >= 0");
    if (ld < c->n) return fail(DMC_E_INVALID, "ld must be at least the chain count");
    if (c->D > 0 && (!flow || !u)) return fail(DMC_E_INVALID, "chains that keep coordinates need a flow and u");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(DMC_E_INVALID, "alpha must be in [0, 1]");
    if (acc->n_groups != c->n_groups || acc->n_k != c->n_k || acc->n_roots != c->n_roots || n_k != c->n_k)
        return fail(DMC_E_INVALID, "the accumulator and the chains must have one observable shape");
    const int64_t n = c->n;
    for (int64_t t = 0; t < thermal + steps; ++t) {
        const uint64_t idx = first + (uint64_t)t * (uint64_t)n;
        dmc_status st = flow ? dmc_flow_sample(flow, s, seed, idx, n, x, ld, jac, c->D > 0 ? u : nullptr, nullptr,
                                               mix_flow, mix_uniform, stream)
                             : dmc_sample(s, seed, idx, n, x, ld, jac, stream);
        if (st != DMC_OK) return st;
        st = dmc_eval_batch(g, inst, n_inst, k_ext, n_k, x, ld, jac, n, acc, f, nullptr, stream);
        if (st != DMC_OK) return st;
        st = dmc_accumulate(acc, nullptr, nullptr, stream);
        if (st != DMC_OK) return st;
        st = chains_step(c, f, n, jac, nullptr, nullptr, c->D > 0 ? u : nullptr, ld, chain_offset(offset_key, t, n),
                         alpha, accept_seed, t >= thermal, stream);
        if (st != DMC_OK) return st;
        if (thermal > 0 && t + 1 == thermal) {
            st = dmc_chains_reset(c, stream);
            if (st != DMC_OK) return st;
        }
    }
    return DMC_OK;
}

void dmc_chains_destroy(dmc_chains* c) {
    if (!c) return;
    (void)hipFree(c->f_state);
    (void)hipFree(c->u_state);
    (void)hipFree(c->q_state);
    (void)hipFree(c->pi_state);
    (void)hipFree(c->partial);
    (void)hipFree(c->totals);
    (void)hipFree(c->zeros);
    (void)hipFree(c->nonfin);
    (void)hipFree(c->n_acc);
    delete c;
}

}  // extern "C"

dmc_status dmc_probe(int32_t kind, int64_t work, double* ms, double* ops, void* stream) {
    if (!ms || !ops) return fail(DMC_E_INVALID, "null argument");
    if (kind < 0 || kind > 3) return fail(DMC_E_INVALID, "kind must be 0 (FMA), 1 (2^x), 2 (reciprocal) or 3 (copy)");
    if (work < 1 || (kind < 3 && work > (1 << 20)) || (kind == 3 && (work % 16 != 0 || work > ((int64_t)1 << 36))))
        return fail(DMC_E_INVALID, "work: iterations in [1, 2^20], or bytes, a multiple of 16, up to 64 GiB");
    const int blocks = 8 * cu_count();
    float *out = nullptr, *in = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dmc_status st = DMC_OK;
    auto done = [&]() {
        (void)hipFree(out);
        (void)hipFree(in);
        (void)hipFree(dst);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return st;
    };
    int64_t n4 = 0;
    if (kind < 3) {
        if (hipMalloc(&out, sizeof(float) * (size_t)blocks * 256) != hipSuccess) {
            st = fail(DMC_E_NOMEM, "probe allocation failed");
            return done();
        }
        *ops = (double)blocks * 256.0 * (double)work * 16.0 * 8.0;
    } else {
        n4 = work / 16;
        if (hipMalloc(&in, (size_t)work) != hipSuccess || hipMalloc(&dst, (size_t)work) != hipSuccess ||
            hipMemsetAsync(in, 0, (size_t)work, S(stream)) != hipSuccess) {
            st = fail(DMC_E_NOMEM, "probe allocation failed");
            return done();
        }
        *ops = 2.0 * (double)work;  // bytes read plus bytes written
    }
    const int it = (int)std::min<int64_t>(work, 1 << 20);
    const int grid = kind < 3 ? blocks : 4 * blocks;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        dmc::launch_probe(kind, out, grid, it, in, dst, n4, S(stream)) != hipSuccess ||  // warm-up
        hipEventRecord(e0, S(stream)) != hipSuccess ||
        dmc::launch_probe(kind, out, grid, it, in, dst, n4, S(stream)) != hipSuccess ||
        hipEventRecord(e1, S(stream)) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = fail(DMC_E_DEVICE, "probe launch failed");
        return done();
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = fail(DMC_E_DEVICE, "probe timing failed");
    *ms = t;
    return done();
}

// ------------------------------------------------------------------------------ checkpoint
// Layout (native byte order): "DMCCKPT1", u64 seed, u64 next_index, u32 sections (1 sampler, 2 flow, 4
// accumulator), then each present section in that order.
//   sampler: i32 kind, order, dim, n_bins; f64 beta, qmax; f64 edges[dim (n_bins + 1)]; f64 hist[dim n_bins]
//   flow:    i32 kind, dim, n_layers, pad; i64 n_params, step; i8 masks[n_layers dim]; f32 master, m, v [n_params]
//   accum:   i32 n_groups, n_k, n_roots, n_inst; i64 n_samples; u64 nonfinite; i32 group[n_inst];
//            f64 factor[n_inst]; f64 totals[2 s_total]
namespace {
struct Writer {
    unsigned char* p;
    size_t cap, len = 0;
    template <class T>
    void put(const T* v, size_t n) {
        const size_t b = sizeof(T) * n;
        if (p && len + b <= cap) std::memcpy(p + len, v, b);
        len += b;
    }
    template <class T>
    void put1(T v) { put(&v, 1); }
};
struct Reader {
    const unsigned char* p;
    size_t len, pos = 0;
    template <class T>
    bool get(T* v, size_t n) {
        const size_t b = sizeof(T) * n;
        if (pos + b > len) return false;
        std::memcpy(v, p + pos, b);
        pos += b;
        return true;
    }
    template <class T>
    bool get1(T& v) { return get(&v, 1); }
};
size_t flow_param_len(const dmc_flow* f) {
    return f->kind == 1 ? (size_t)f->n_params : (size_t)f->n_layers * dmc::LAYER_SIZE;
}
}  // namespace

extern "C" {

dmc_status dmc_checkpoint_save(const dmc_sampler* s, const dmc_flow* f, const dmc_accum* acc, uint64_t seed,
                               uint64_t next_index, void* buf, size_t cap, size_t* len, void* stream) {
    if (!len) return fail(DMC_E_INVALID, "null length");
    if (acc && acc->pending_blocks) return fail(DMC_E_STATE, "an evaluation is waiting for dmc_accumulate");
    if (s || f || acc) HIP_TRY(hipStreamSynchronize(S(stream)));
    Writer w{static_cast<unsigned char*>(buf), buf ? cap : 0};
    w.put("DMCCKPT1", 8);
    w.put1(seed);
    w.put1(next_index);
    w.put1((uint32_t)((s ? 1 : 0) | (f ? 2 : 0) | (acc ? 4 : 0)));
    if (s) {
        const int32_t hdr[4] = {s->kind, s->order, s->dim, s->n_bins};
        w.put(hdr, 4);
        w.put1(s->beta);
        w.put1(s->qmax);
        w.put(s->edges.data(), s->edges.size());
        std::vector<double> h((size_t)s->dim * s->n_bins);
        HIP_TRY(hipMemcpy(h.data(), s->d_hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        w.put(h.data(), h.size());
    }
    if (f) {
        const int32_t hdr[4] = {f->kind, f->dim, f->n_layers, 0};
        w.put(hdr, 4);
        const size_t P = flow_param_len(f);
        w.put1((int64_t)P);
        w.put1(f->step);
        w.put(f->masks.data(), f->masks.size());
        std::vector<float> t(P);
        for (float* src : {f->master, f->m, f->v}) {
            HIP_TRY(hipMemcpy(t.data(), src, sizeof(float) * P, hipMemcpyDeviceToHost));
            w.put(t.data(), P);
        }
    }
    if (acc) {
        const int32_t hdr[4] = {acc->n_groups, acc->n_k, acc->n_roots, (int32_t)acc->inst_group.size()};
        w.put(hdr, 4);
        w.put1(acc->n_samples);
        unsigned long long nf = 0;
        HIP_TRY(hipMemcpy(&nf, acc->nonfin_tot, sizeof(nf), hipMemcpyDeviceToHost));
        w.put1((uint64_t)nf);
        w.put(acc->inst_group.data(), acc->inst_group.size());
        w.put(acc->inst_factor.data(), acc->inst_factor.size());
        std::vector<double> t(2 * (size_t)acc->s_total);
        HIP_TRY(hipMemcpy(t.data(), acc->totals, sizeof(double) * t.size(), hipMemcpyDeviceToHost));
        w.put(t.data(), t.size());
    }
    *len = w.len;
    if (buf && w.len > cap) return fail(DMC_E_INVALID, "buffer too small for the checkpoint");
    return DMC_OK;
}

dmc_status dmc_checkpoint_load(dmc_sampler* s, dmc_flow* f, dmc_accum* acc, uint64_t* seed, uint64_t* next_index,
                               const void* buf, size_t len, void* stream) {
    if (!buf) return fail(DMC_E_INVALID, "null buffer");
    Reader r{static_cast<const unsigned char*>(buf), len};
    char magic[8];
    uint64_t sd = 0, nx = 0;
    uint32_t sec = 0;
    if (!r.get(magic, 8) || std::memcmp(magic, "DMCCKPT1", 8) != 0 || !r.get1(sd) || !r.get1(nx) || !r.get1(sec))
        return fail(DMC_E_INVALID, "not a checkpoint");
    if ((s && !(sec & 1)) || (f && !(sec & 2)) || (acc && !(sec & 4)))
        return fail(DMC_E_INVALID, "the checkpoint lacks a section for a handle passed");
    if (acc && acc->pending_blocks) return fail(DMC_E_STATE, "an evaluation is waiting for dmc_accumulate");
    // parse everything first, so that a malformed or mismatching checkpoint changes no handle
    std::vector<double> edges, hist, totals, factor;
    std::vector<float> fm, fmm, fv;
    std::vector<int32_t> group;
    std::vector<int8_t> masks;
    int64_t fstep = 0, n_samples = 0;
    uint64_t nonfin = 0;
    if (sec & 1) {
        int32_t h[4];
        double beta, qmax;
        if (!r.get(h, 4) || !r.get1(beta) || !r.get1(qmax)) return fail(DMC_E_INVALID, "truncated checkpoint");
        if (h[2] < 1 || h[3] < 1 || h[2] > 64 || h[3] > 4096) return fail(DMC_E_INVALID, "corrupt sampler section");
        edges.resize((size_t)h[2] * (h[3] + 1));
        hist.resize((size_t)h[2] * h[3]);
        if (!r.get(edges.data(), edges.size()) || !r.get(hist.data(), hist.size()))
            return fail(DMC_E_INVALID, "truncated checkpoint");
        if (s && (h[0] != s->kind || h[1] != s->order || h[2] != s->dim || h[3] != s->n_bins || beta != s->beta ||
                  qmax != s->qmax))
            return fail(DMC_E_INVALID, "the sampler does not match the checkpoint");
    }
    if (sec & 2) {
        int32_t h[4];
        int64_t P = 0;
        if (!r.get(h, 4) || !r.get1(P) || !r.get1(fstep)) return fail(DMC_E_INVALID, "truncated checkpoint");
        if (h[1] < 1 || h[1] > 64 || h[2] < 1 || h[2] > 64 || P < 1 || P > (int64_t)1 << 28)
            return fail(DMC_E_INVALID, "corrupt flow section");
        masks.resize((size_t)h[2] * h[1]);
        fm.resize(P);
        fmm.resize(P);
        fv.resize(P);
        if (!r.get(masks.data(), masks.size()) || !r.get(fm.data(), P) || !r.get(fmm.data(), P) || !r.get(fv.data(), P))
            return fail(DMC_E_INVALID, "truncated checkpoint");
        if (f && (h[0] != f->kind || h[1] != f->dim || h[2] != f->n_layers || (size_t)P != flow_param_len(f) ||
                  masks != f->masks))
            return fail(DMC_E_INVALID, "the flow does not match the checkpoint");
    }
    if (sec & 4) {
        int32_t h[4];
        if (!r.get(h, 4) || !r.get1(n_samples) || !r.get1(nonfin)) return fail(DMC_E_INVALID, "truncated checkpoint");
        if (h[0] < 1 || h[0] > DMC_MAX_GROUPS || h[1] < 1 || h[1] > DMC_MAX_K || h[2] < 1 || h[2] > DMC_MAX_ROOTS ||
            h[3] < 0 || h[3] > DMC_MAX_INSTANCES)
            return fail(DMC_E_INVALID, "corrupt accumulator section");
        group.resize(h[3]);
        factor.resize(h[3]);
        totals.resize(2 * (size_t)h[1] * 2 * h[0] * h[2]);
        if (!r.get(group.data(), group.size()) || !r.get(factor.data(), factor.size()) ||
            !r.get(totals.data(), totals.size()))
            return fail(DMC_E_INVALID, "truncated checkpoint");
        if (acc && (h[0] != acc->n_groups || h[1] != acc->n_k || h[2] != acc->n_roots))
            return fail(DMC_E_INVALID, "the accumulator does not match the checkpoint");
    }
    if (s || f || acc) HIP_TRY(hipStreamSynchronize(S(stream)));
    if (s) {
        s->edges = edges;
        std::vector<float> ef(edges.begin(), edges.end());
        HIP_TRY(hipMemcpy(s->d_edges, ef.data(), sizeof(float) * ef.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_hist, hist.data(), sizeof(double) * hist.size(), hipMemcpyHostToDevice));
        s->last_n = -1;
    }
    if (f) {
        const size_t P = fm.size();
        HIP_TRY(hipMemcpy(f->master, fm.data(), sizeof(float) * P, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(f->m, fmm.data(), sizeof(float) * P, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(f->v, fv.data(), sizeof(float) * P, hipMemcpyHostToDevice));
        f->step = fstep;
        if (f->kind == 0) HIP_TRY(dmc::launch_flow_shadow(f->master, f->shadow, f->n_layers, cu_count(), S(stream)));
    }
    if (acc) {
        HIP_TRY(hipMemcpy(acc->totals, totals.data(), sizeof(double) * totals.size(), hipMemcpyHostToDevice));
        const unsigned long long nf = nonfin;
        HIP_TRY(hipMemcpy(acc->nonfin_tot, &nf, sizeof(nf), hipMemcpyHostToDevice));
        acc->n_samples = n_samples;
        acc->inst_group.assign(group.begin(), group.end());
        acc->inst_factor.assign(factor.begin(), factor.end());
    }
    if (seed) *seed = sd;
    if (next_index) *next_index = nx;
    if (s || f || acc) HIP_TRY(hipStreamSynchronize(S(stream)));
    return DMC_OK;
}

}  // extern "C"
