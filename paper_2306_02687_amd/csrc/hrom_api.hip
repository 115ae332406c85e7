// C ABI of the hyper-reduced RVE library: plan creation (device layouts and
// workspace), and the evaluate / condense / update / backward entry points,
// which only enqueue kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <type_traits>

#include "hrom_internal.h"

using namespace hrom;

struct hrom_plan_s {
    Plan p;
};

namespace {

template <typename T>
int dalloc(T** ptr, int64_t n) {
    *ptr = nullptr;
    if (n <= 0) n = 1;
    if (hipMalloc((void**)ptr, sizeof(T) * (size_t)n) != hipSuccess) {
        *ptr = nullptr;
        return HROM_E_NOMEM;
    }
    return HROM_OK;
}

template <typename T>
void dfree(T*& ptr) {
    if (ptr) (void)hipFree((void*)ptr);
    ptr = nullptr;
}

void free_plan(Plan& p) {
    if (p.owns_arena) dfree(p.arena);
    p.arena = nullptr;
    dfree(p.cls_dev); dfree(p.items_tan); dfree(p.counter);
}

int hip_status() { return hipGetLastError() == hipSuccess ? HROM_OK : HROM_E_HIP; }

bool mixed(const Plan& p) { return p.prec != HROM_FP64; }

// iterative refinement of the adjoint solve (mixed plans that ask for it)
bool refine(const Plan& p) { return mixed(p) && (p.flags & HROM_REFINE); }

// ECM-weight part of the power-of-two scaling of w_q A_q for the low-precision
// operands (w ~ 1/Q); the material part comes from theta on the device
int qexp_for(int Q) { return (int)std::ceil(std::log2((double)Q)); }

template <typename T>
int upload(T** dst, const std::vector<T>& v) {
    int rc = dalloc(dst, (int64_t)v.size());
    if (rc == HROM_OK && !v.empty() &&
        hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        rc = HROM_E_HIP;
    return rc;
}

// Validates the cluster descriptors and fills the plan's cluster geometry and
// offsets (host only, no device access, no allocation beyond p.cl's
// reserved capacity).
int plan_geometry(Plan& p, const hrom_cluster* clusters, int32_t ncl, int64_t N, int32_t precision,
                  uint32_t flags) {
    if (!clusters || ncl < 1 || N < 1) return HROM_E_INVALID;
    if (precision != HROM_FP64 && precision != HROM_MIXED_BF16 && precision != HROM_MIXED_FP16)
        return HROM_E_INVALID;
    // a single low-precision term per product misses the 1e-5 accuracy of the
    // mixed path (and makes Kaa indefinite when some modes are soft)
    if (precision != HROM_FP64 && !(flags & HROM_SPLIT)) return HROM_E_UNSUPPORTED;
    // the six-component condensation condenses the symmetric stretch of the objective split
    if ((flags & HROM_BIOT6) && !(flags & HROM_OBJECTIVE)) return HROM_E_UNSUPPORTED;
    int64_t next = 0;
    for (int c = 0; c < ncl; c++) {
        const hrom_cluster& k = clusters[c];
        if (!k.G || !k.w || !k.phase || k.Q < 1 || k.count < 1 || k.first != next) return HROM_E_INVALID;
        if (k.m < 1 || k.m > kMaxModes) return HROM_E_UNSUPPORTED;
        next += k.count;
    }
    if (next != N) return HROM_E_INVALID;
    p.ncl = ncl;
    p.N = N;
    p.prec = precision;
    p.flags = flags;
    p.j2 = (flags & HROM_J2) != 0;
    p.nmac = (flags & HROM_BIOT6) ? 6 : 9;
    p.cl.clear();
    int64_t off_a = 0, off_kaa = 0, off_kaf = 0, ws_k = 0, ws_L = 0, ws_q = 0, ws_h = 0;
    for (int c = 0; c < ncl; c++) {
        const hrom_cluster& k = clusters[c];
        ClusterDev d{};
        d.m = k.m;
        d.Q = k.Q;
        d.Qpad = (k.Q + 63) / 64 * 64;
        d.MT = (k.m + 10 + 15) / 16;
        d.MP = 16 * d.MT;
        d.res_t = (k.m + 9) / 16;
        d.res_c = (k.m + 9) % 16;
        d.KS = 4 * ((k.m + 15) / 16);   // k-steps padded to whole mode tiles (zeros beyond m)
        d.first = k.first;
        d.count = k.count;
        d.off_a = off_a;
        d.off_kaa = off_kaa;
        d.off_kaf = off_kaf;
        d.ws_khat = ws_k;
        d.ws_L = ws_L;
        d.ws_qs = ws_q;
        d.ws_hist = ws_h;
        if (p.j2) ws_h += (int64_t)8 * d.Qpad * k.count;
        off_a += (int64_t)k.m * k.count;
        off_kaa += (int64_t)k.m * k.m * k.count;
        off_kaf += (int64_t)9 * k.m * k.count;
        ws_k += khat_len(d.m, d.MT, precision != HROM_FP64) * k.count;
        ws_L += (int64_t)k.m * k.m * k.count;
        ws_q += (int64_t)12 * d.Qpad * k.count;
        p.cl.push_back(d);
    }
    p.a_len = off_a;
    p.kaa_len = off_kaa;
    p.kaf_len = off_kaf;
    p.khat_len = ws_k;
    p.L_len = ws_L;
    p.qs_len = ws_q;
    p.hist_len = ws_h;
    return HROM_OK;
}

// Carves every device buffer of the plan out of one region starting at base
// (256-byte aligned pieces, in a fixed order) and returns the region's size;
// with base == nullptr only the size is computed.
size_t plan_carve(Plan& p, char* base) {
    size_t off = 0;
    auto take = [&](auto*& ptr, int64_t n) {
        using T = std::remove_reference_t<decltype(*ptr)>;
        if (n < 1) n = 1;
        off = (off + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)n;
    };
    const bool mx = mixed(p);
    for (auto& d : p.cl) {
        take(d.Ghat, (int64_t)d.Qpad * 9 * d.MP);
        take(d.GT, (int64_t)d.Qpad * 9 * d.m);
        take(d.Gf, (int64_t)d.Qpad * 9 / 16 * d.KS * 64);
        take(d.w, d.Qpad);
        take(d.phase, d.Qpad);
        if (mx) {
            take(d.Fpk, (int64_t)d.Qpad * ((d.m + 15) / 16) * 512);
            take(d.Gb3, (int64_t)d.Qpad * 9 / 16 * gb3_halves(d.m) * 3 * 64 * 4);
        } else {
            d.Fpk = nullptr;
            d.Gb3 = nullptr;
        }
        take(d.gram, (int64_t)d.m * d.m);
        take(d.gram_part, (int64_t)((d.Q + kGramChunk - 1) / kGramChunk) * d.m * d.m);
        take(d.R, (int64_t)d.m * d.m);
        take(d.Rinv, (int64_t)d.m * d.m);
        take(d.Gt, (int64_t)d.Q * 9 * d.m);
        take(d.kscale, 1);
    }
    take(p.basis_flag, 1);
    if (p.j2) {
        take(p.hist_n, p.hist_len);
        take(p.hist_t, p.hist_len);
    } else {
        p.hist_n = p.hist_t = nullptr;
    }
    take(p.at, p.a_len);
    take(p.dt, p.a_len);
    const int64_t n = p.N;
    take(p.Fr, 9 * n);
    take(p.polar, 21 * n);
    take(p.Pr, 9 * n);
    take(p.r, p.a_len);
    if (mx) {
        float* kh; take(kh, p.khat_len); p.Khat = kh;
        float* qs; take(qs, p.qs_len); p.qs = qs;
    } else {
        double* kh; take(kh, p.khat_len); p.Khat = kh;
        double* qs; take(qs, p.qs_len); p.qs = qs;
    }
    take(p.L, refine(p) ? p.L_len : 1);
    take(p.piv, p.a_len);
    take(p.y, p.a_len);
    take(p.X, (int64_t)p.nmac * p.a_len);
    take(p.Palg, 9 * n);
    take(p.Cr, 81 * n);
    take(p.S, 9 * n);
    take(p.rnorm, n);
    take(p.dU, 9 * n);
    take(p.gr, 9 * n);
    take(p.Lam, 9 * n);
    take(p.lam, p.a_len);
    take(p.rho, p.a_len);
    take(p.conv, n);
    take(p.hr, 9 * n);
    take(p.gth, 4 * n);
    take(p.gth_part, 4 * kThetaChunks);
    return (off + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// Enqueues the build of every cluster's device layouts (Ghat, GT, Gf, the
// packed low-precision fragments, padded w and phase) from the caller's G, w,
// phase on stream s.
void plan_build(const Plan& p, const hrom_cluster* clusters, hipStream_t s) {
    for (int c = 0; c < p.ncl; c++) {
        const hrom_cluster& k = clusters[c];
        const ClusterDev& d = p.cl[c];
        BasisArgs ba{d.m, d.Q, k.G, k.w, d.gram, d.gram_part, d.R, d.Rinv, d.Gt, p.basis_flag};
        launch_basis_build(ba, s);
        LayoutArgs la{};
        la.m = d.m; la.Q = d.Q; la.Qpad = d.Qpad; la.MT = d.MT; la.MP = d.MP; la.prec = p.prec;
        la.G = d.Gt; la.w = k.w; la.phase = k.phase;
        la.Ghat = d.Ghat; la.GT = d.GT; la.Gf = d.Gf; la.KS = d.KS; la.wpad = d.w; la.phpad = d.phase;
        la.Fpk = d.Fpk; la.Gb3 = d.Gb3; la.split = (p.flags & HROM_SPLIT) ? 1 : 0;
        launch_build_layouts(la, s);
    }
}

// Device cluster table and the cost-sorted work queues of the tangent launches.
int build_groups(Plan& p) {
    p.grouped = p.ncl > 1 && !p.j2;   // J2 plans: the FP64 tangent per cluster
    std::vector<ClusterGPU> cg;
    std::vector<WorkItem> tan;
    p.max_m = 0;
    for (int c = 0; c < p.ncl; c++) {
        const ClusterDev& d = p.cl[c];
        ClusterGPU g{};
        g.m = d.m; g.Q = d.Q; g.Qpad = d.Qpad; g.MP = d.MP; g.MT = d.MT; g.KS = d.KS;
        g.first = d.first; g.count = d.count; g.off_a = d.off_a; g.ws_qs = d.ws_qs;
        g.ws_khat = d.ws_khat; g.ws_L = d.ws_L;
        g.Ghat = d.Ghat; g.Gf = d.Gf; g.w = d.w; g.phase = d.phase; g.Fpk = d.Fpk;
        cg.push_back(g);
        p.max_m = std::max(p.max_m, d.m);
        // FP64 plans: the persistent tangent launch takes 4-point tiles
        if (!mixed(p))
            for (int64_t u = 0; u < (d.count + 3) / 4; u++) tan.push_back(WorkItem{c, (int)u});
    }
    // most expensive tiles first: tangent ~ MT^2 Q
    auto cost_tan = [&](const WorkItem& w) {
        const double mt = p.cl[w.c].MT;
        return mt * (mt + 1) * p.cl[w.c].Q;
    };
    std::stable_sort(tan.begin(), tan.end(),
                     [&](const WorkItem& x, const WorkItem& y) { return cost_tan(x) > cost_tan(y); });
    p.n_tan = (int)tan.size();
    int ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p.device) == hipSuccess && prop.multiProcessorCount > 0)
        ncu = prop.multiProcessorCount;
    p.persistent_grid = std::min(p.n_tan, 2 * ncu);
    int rc = upload(&p.cls_dev, cg);
    if (rc == HROM_OK) rc = upload(&p.items_tan, tan);
    if (rc == HROM_OK) rc = dalloc(&p.counter, 1);
    return rc;
}

// the caller's amplitudes in the plan's mode basis: at = R a, per cluster
void map_in(const Plan& p, const double* a, hipStream_t s) {
    for (const auto& c : p.cl) {
        ModeMapArgs ma{c.m, c.first, c.count, c.R, a + c.off_a, p.at + c.off_a, nullptr};
        launch_mode_map(MAP_R, ma, s);
    }
}

GroupCall group_call(const Plan& p) {
    GroupCall g{};
    g.cls = p.cls_dev;
    g.ncl = p.ncl;
    g.N = p.N;
    g.counter = p.counter;
    return g;
}

}  // namespace

extern "C" {

const char* hrom_strerror(int code) {
    switch (code) {
        case HROM_OK: return "ok";
        case HROM_E_INVALID: return "invalid argument";
        case HROM_E_HIP: return "HIP runtime error";
        case HROM_E_ORDER: return "call order violated (evaluate before condense, condense before update/backward)";
        case HROM_E_NOMEM: return "device allocation failed";
        case HROM_E_UNSUPPORTED: return "not supported (size outside the supported range, or an output the plan's mode does not provide)";
        case HROM_E_SCRATCH: return "the request needs more device memory than the static scratch of the allocation-free entry point";
        case HROM_E_NOCONV: return "an iteration did not reach its tolerance (SVD sweeps, NNLS)";
        case HROM_E_RANK: return "rank deficiency (truncation beyond the rank of the training matrix, or a dependent column)";
        default: return "unknown error";
    }
}

int hrom_plan_create(hrom_plan* out, const hrom_cluster* clusters, int32_t ncl, int64_t N,
                     int32_t precision, uint32_t flags) {
    if (!out) return HROM_E_INVALID;
    *out = nullptr;
    hrom_plan_s* h = new (std::nothrow) hrom_plan_s;
    if (!h) return HROM_E_NOMEM;
    Plan& p = h->p;
    int rc = plan_geometry(p, clusters, ncl, N, precision, flags);
    if (rc != HROM_OK) {
        delete h;
        return rc;
    }
    (void)hipGetDevice(&p.device);
    const size_t bytes = plan_carve(p, nullptr);
    p.owns_arena = true;
    if (hipMalloc((void**)&p.arena, bytes) != hipSuccess) {
        p.arena = nullptr;
        rc = HROM_E_NOMEM;
    }
    if (rc == HROM_OK) {
        set_kernel_attributes();
        rc = set_basis_attributes();
    }
    if (rc == HROM_OK) {
        p.arena_bytes = bytes;
        plan_carve(p, p.arena);
        if (hipMemset(p.basis_flag, 0, sizeof(int)) != hipSuccess) rc = HROM_E_HIP;
        // J2: virgin material (no plastic strain) in both history buffers
        if (rc == HROM_OK && p.j2 &&
            (hipMemset(p.hist_n, 0, sizeof(double) * p.hist_len) != hipSuccess ||
             hipMemset(p.hist_t, 0, sizeof(double) * p.hist_len) != hipSuccess))
            rc = HROM_E_HIP;
        if (rc == HROM_OK) plan_build(p, clusters, nullptr);
        if (rc == HROM_OK && hipDeviceSynchronize() != hipSuccess) rc = HROM_E_HIP;
        int bad = 0;
        if (rc == HROM_OK && hipMemcpy(&bad, p.basis_flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            rc = HROM_E_HIP;
        // mode gradients linearly dependent in the weighted inner product:
        // Kaa would be singular at every macro point
        if (rc == HROM_OK && bad) rc = HROM_E_INVALID;
    }
    if (rc == HROM_OK) rc = build_groups(p);
    if (rc != HROM_OK) {
        free_plan(p);
        delete h;
        return rc;
    }
    *out = h;
    return HROM_OK;
}

int32_t hrom_num_variants(void) { return 6; }

int32_t hrom_num_kernel_variants(int32_t kind) {
    switch (kind) {
        case HROM_VK_TANGENT: return hrom_num_variants();
        case HROM_VK_KIN: return 2;
        case HROM_VK_CONDENSE: return 2;
        default: return 0;
    }
}

int hrom_plan_set_kernel_variant(hrom_plan plan, int32_t kind, int32_t c, int32_t variant) {
    if (kind == HROM_VK_TANGENT) return hrom_plan_set_variant(plan, c, variant);
    if (!plan || variant < 0 || variant >= hrom_num_kernel_variants(kind) || c < -1 || c >= plan->p.ncl)
        return HROM_E_INVALID;
    Plan& p = plan->p;
    for (int k = 0; k < p.ncl; k++) {
        if (c >= 0 && c != k) continue;
        if (kind == HROM_VK_KIN) p.cl[k].kin_variant = variant;
        else p.cl[k].cond_variant = variant;
    }
    return HROM_OK;
}

int hrom_plan_set_variant(hrom_plan plan, int32_t c, int32_t variant) {
    if (!plan || variant < 0 || variant >= hrom_num_variants() || c < -1 || c >= plan->p.ncl) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.grouped && !mixed(p)) {
        // FP64 with several clusters: one persistent launch for every
        // cluster, the variant picks its grid
        int ncu = 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p.device) == hipSuccess && prop.multiProcessorCount > 0)
            ncu = prop.multiProcessorCount;
        p.persistent_grid = std::min(p.n_tan, (variant + 1) * ncu);
        return HROM_OK;
    }
    for (int k = 0; k < p.ncl; k++)
        if (c < 0 || c == k) p.cl[k].variant = variant;
    return HROM_OK;
}

int hrom_plan_destroy(hrom_plan plan) {
    if (!plan) return HROM_E_INVALID;
    (void)hipDeviceSynchronize();
    for (auto& e : plan->p.ev_tan)
        if (e) (void)hipEventDestroy(e);
    free_plan(plan->p);
    delete plan;
    return HROM_OK;
}

int hrom_plan_profile(hrom_plan plan, int32_t enable) {
    if (!plan) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (enable && !p.ev_tan[0]) {
        if (hipEventCreate(&p.ev_tan[0]) != hipSuccess || hipEventCreate(&p.ev_tan[1]) != hipSuccess)
            return HROM_E_HIP;
    }
    p.profile = enable != 0;
    return HROM_OK;
}

int hrom_plan_tangent_ms(hrom_plan plan, float* ms) {
    if (!plan || !ms) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (!p.profile) return HROM_E_ORDER;
    if (hipEventSynchronize(p.ev_tan[1]) != hipSuccess) return HROM_E_HIP;
    return hipEventElapsedTime(ms, p.ev_tan[0], p.ev_tan[1]) == hipSuccess ? HROM_OK : HROM_E_HIP;
}

int64_t hrom_plan_offset(hrom_plan plan, int32_t c, int32_t kind) {
    if (!plan || c < 0 || c > plan->p.ncl) return -1;
    const Plan& p = plan->p;
    if (c == p.ncl) {
        if (kind == HROM_OFF_A) return p.a_len;
        if (kind == HROM_OFF_KAA) return p.kaa_len;
        if (kind == HROM_OFF_KAF) return p.kaf_len;
        return -1;
    }
    if (kind == HROM_OFF_A) return p.cl[c].off_a;
    if (kind == HROM_OFF_KAA) return p.cl[c].off_kaa;
    if (kind == HROM_OFF_KAF) return p.cl[c].off_kaf;
    return -1;
}

int hrom_eval(hrom_plan plan, const double* theta, const double* Fbar, const double* a, double* r,
              double* Pr, double* Kaa, double* KaF, double* KFF, int32_t* status, hipStream_t stream) {
    if (!plan || !theta || !Fbar || !a || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    PointArgs pa{p.N, (p.flags & HROM_OBJECTIVE) ? 1 : 0, Fbar, p.Fr, p.polar, status};
    launch_prepare(pa, stream);
    map_in(p, a, stream);
    const size_t tsz = mixed(p) ? sizeof(float) : sizeof(double);
    std::vector<EvalArgs> tan_args;   // per-cluster tangent launches of a mixed plan with several clusters
    for (const auto& c : p.cl) {
        EvalArgs e{};
        e.m = c.m; e.Q = c.Q; e.Qpad = c.Qpad; e.MP = c.MP; e.MT = c.MT; e.KS = c.KS;
        e.first = c.first; e.count = c.count; e.N = p.N;
        e.Ghat = c.Ghat; e.Gf = c.Gf; e.w = c.w; e.phase = c.phase; e.Fpk = c.Fpk;
        e.theta = theta; e.Fr = p.Fr; e.a = p.at + c.off_a;
        e.qs = (char*)p.qs + tsz * (size_t)c.ws_qs;
        e.Khat = (char*)p.Khat + tsz * (size_t)c.ws_khat;
        e.r = p.r + c.off_a;
        e.Pr = p.Pr;
        e.status = status;
        e.qexp = qexp_for(c.Q);
        e.kscale_out = c.kscale;
        e.hist_n = p.j2 ? p.hist_n + c.ws_hist : nullptr;
        e.hist_t = p.j2 ? p.hist_t + c.ws_hist : nullptr;
        int rc = launch_kin(mixed(p) ? 1 : 0, p.j2 ? 1 : 0, c.kin_variant, e, stream);
        if (rc != HROM_OK) return rc;
        if (p.grouped) {
            tan_args.push_back(e);
            continue;
        }
        // single-cluster plans: the events bracket the (only) tangent launch
        if (p.profile) (void)hipEventRecord(p.ev_tan[0], stream);
        rc = mixed(p) ? launch_eval_mixed(c.MT, p.prec, (p.flags & HROM_SPLIT) != 0, c.variant, p.j2 ? 1 : 0, e,
                                          stream)
                      : launch_eval_f64(c.MT, c.variant, p.j2 ? 1 : 0, e, stream);
        if (p.profile) (void)hipEventRecord(p.ev_tan[1], stream);
        if (rc != HROM_OK) return rc;
    }
    if (p.grouped) {
        // several clusters, after all kinematics launches: FP64 plans run the
        // tangent contraction of every cluster in one persistent launch over a
        // cost-sorted work queue; mixed plans launch it once per cluster, each
        // at the occupancy its mode count allows
        int rc = HROM_OK;
        if (p.profile) (void)hipEventRecord(p.ev_tan[0], stream);
        if (!mixed(p)) {
            GroupCall g = group_call(p);
            g.theta = theta; g.Fr = p.Fr; g.a = p.at; g.qs = p.qs; g.Khat = p.Khat;
            g.r = p.r; g.Pr = p.Pr; g.status = status;
            g.items = p.items_tan; g.nitems = p.n_tan;
            rc = launch_tan_persistent(g, p.persistent_grid, stream);
        } else {
            for (int k = 0; k < p.ncl && rc == HROM_OK; k++)
                rc = launch_eval_mixed(p.cl[k].MT, p.prec, (p.flags & HROM_SPLIT) != 0, p.cl[k].variant, 0,
                                       tan_args[k], stream);
        }
        if (p.profile) (void)hipEventRecord(p.ev_tan[1], stream);
        if (rc != HROM_OK) return rc;
    }
    if (Kaa || KaF || KFF) {
        for (const auto& c : p.cl) {
            CondenseArgs ca{};
            ca.m = c.m; ca.MT = c.MT; ca.res_t = c.res_t; ca.res_c = c.res_c; ca.mixed = mixed(p);
        ca.nmac = p.nmac;
            ca.first = c.first; ca.count = c.count; ca.N = p.N;
            ca.Khat = (const char*)p.Khat + tsz * (size_t)c.ws_khat;
            ca.r = p.r + c.off_a; ca.Pr = p.Pr;
            ca.kscale = c.kscale;
            ca.outKaa = Kaa ? Kaa + c.off_kaa : nullptr;
            ca.outKaF = KaF ? KaF + c.off_kaf : nullptr;
            ca.outKFF = KFF;
            const int rc = launch_unpack_condense(ca, 0, stream);
            if (rc != HROM_OK) return rc;
            launch_export_basis(c.R, c.m, c.count, ca.outKaa, ca.outKaF, stream);
        }
    }
    if (r) {
        for (const auto& c : p.cl) {
            ModeMapArgs ma{c.m, c.first, c.count, c.R, p.r + c.off_a, r + c.off_a, nullptr};
            launch_mode_map(MAP_RT, ma, stream);
        }
    }
    if (Pr) (void)hipMemcpyAsync(Pr, p.Pr, sizeof(double) * 9 * p.N, hipMemcpyDeviceToDevice, stream);
    const int rc = hip_status();
    if (rc == HROM_OK) p.stage = 1;
    return rc;
}

int hrom_condense(hrom_plan plan, double* Pbar, double* Cbar, double* rnorm, int32_t* status,
                  hipStream_t stream) {
    if (!plan || !Pbar || !Cbar || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.stage < 1) return HROM_E_ORDER;
    const size_t tsz = mixed(p) ? sizeof(float) : sizeof(double);
    for (const auto& c : p.cl) {
        CondenseArgs ca{};
        ca.m = c.m; ca.MT = c.MT; ca.res_t = c.res_t; ca.res_c = c.res_c; ca.mixed = mixed(p);
        ca.nmac = p.nmac;
        ca.first = c.first; ca.count = c.count; ca.N = p.N;
        ca.Khat = (const char*)p.Khat + tsz * (size_t)c.ws_khat;
        ca.r = p.r + c.off_a; ca.Pr = p.Pr;
        ca.L = refine(p) ? p.L + c.ws_L : nullptr;
        ca.piv = p.piv + c.off_a;
        ca.y = p.y + c.off_a; ca.X = p.X + (int64_t)p.nmac * c.off_a;
        ca.Palg = p.Palg; ca.Cr = p.Cr; ca.rnorm = p.rnorm; ca.status = status;
        ca.kscale = c.kscale;
        ca.variant = c.cond_variant;
        // SPD path: register-resident elimination, one launch per cluster so
        // that each runs at the occupancy its mode count allows; non-positive
        // pivots finish on the LU path
        int rc = launch_condense_reg(ca, stream);
        if (rc == HROM_OK) rc = launch_unpack_condense(ca, 2, stream);
        if (rc != HROM_OK) return rc;
        // ||r||_2 in the caller's basis, r = R^T rt
        ModeMapArgs ma{c.m, c.first, c.count, c.R, p.r + c.off_a, nullptr, p.rnorm};
        launch_mode_map(MAP_RT, ma, stream);
    }
    PushArgs pa{p.N, (p.flags & HROM_OBJECTIVE) ? 1 : 0, p.polar, p.Palg, p.Cr, Pbar, Cbar, p.S, status};
    launch_pushout(pa, stream);
    if (rnorm) (void)hipMemcpyAsync(rnorm, p.rnorm, sizeof(double) * p.N, hipMemcpyDeviceToDevice, stream);
    const int rc = hip_status();
    if (rc == HROM_OK) p.stage = 2;
    return rc;
}

}  // extern "C"

static int update_impl(Plan& p, const double* dFbar, double tol, double* a, const int* status,
                       hipStream_t stream) {
    UpdateArgs u{};
    u.N = p.N;
    u.objective = (p.flags & HROM_OBJECTIVE) ? 1 : 0;
    u.dFbar = dFbar;
    u.polar = p.polar;
    u.dU = p.dU;
    u.rnorm = p.rnorm;
    u.status = status;
    u.tol = tol;
    launch_stretch_increment(u, stream);
    for (const auto& c : p.cl) {
        u.m = c.m;
        u.first = c.first;
        u.count = c.count;
        u.y = p.y + c.off_a;
        u.X = p.X + (int64_t)p.nmac * c.off_a;
        u.nmac = p.nmac;
        u.dt = p.dt + c.off_a;
        launch_update(u, stream);
        ModeMapArgs ma{c.m, c.first, c.count, c.Rinv, p.dt + c.off_a, a + c.off_a, nullptr};
        launch_mode_map(MAP_RINV, ma, stream);
    }
    return hip_status();
}

extern "C" {

int hrom_update(hrom_plan plan, const double* dFbar, double tol, double* a, const int32_t* status,
                hipStream_t stream) {
    if (!plan || !a || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.stage < 2) return HROM_E_ORDER;
    const int rc = update_impl(p, dFbar, tol, a, status, stream);
    if (rc == HROM_OK) p.stage = 0;
    return rc;
}

int hrom_newton(hrom_plan plan, const double* theta, const double* Fbar, double* a, double tol,
                int32_t max_it, double* Pbar, double* Cbar, double* rnorm, int32_t* status,
                hipStream_t stream) {
    if (!plan || max_it < 1) return HROM_E_INVALID;
    int rc = HROM_OK;
    for (int it = 0; it < max_it && rc == HROM_OK; it++) {
        rc = hrom_eval(plan, theta, Fbar, a, nullptr, nullptr, nullptr, nullptr, nullptr, status, stream);
        if (rc == HROM_OK) rc = hrom_condense(plan, Pbar, Cbar, rnorm, status, stream);
        if (rc == HROM_OK && it + 1 < max_it) {
            rc = update_impl(plan->p, nullptr, tol, a, status, stream);
            // the state of the last evaluation stays valid for the frozen points only;
            // the next iteration re-evaluates every point
        }
    }
    if (rc == HROM_OK) {
        launch_mark_unconverged(plan->p.N, plan->p.rnorm, tol, status, stream);
        rc = hip_status();
    }
    return rc;
}

int hrom_biot(hrom_plan plan, double* T, double* CB, int32_t* status, hipStream_t stream) {
    if (!plan || !T || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.stage < 2) return HROM_E_ORDER;
    if (!(p.flags & HROM_OBJECTIVE)) return HROM_E_UNSUPPORTED;
    BiotArgs ba{p.N, p.Palg, p.Cr, T, CB, status};
    launch_biot(ba, stream);
    return hip_status();
}

int hrom_commit(hrom_plan plan, hipStream_t stream) {
    if (!plan) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (!p.j2) return HROM_E_UNSUPPORTED;
    if (p.stage < 1) return HROM_E_ORDER;
    if (hipMemcpyAsync(p.hist_n, p.hist_t, sizeof(double) * p.hist_len, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess)
        return HROM_E_HIP;
    return HROM_OK;
}

int hrom_history(hrom_plan plan, int32_t which, double* out, hipStream_t stream) {
    if (!plan || !out || (which != 0 && which != 1)) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (!p.j2) return HROM_E_UNSUPPORTED;
    int64_t off = 0;
    for (const auto& c : p.cl) {
        const double* src = (which ? p.hist_t : p.hist_n) + c.ws_hist;
        launch_history_export(src, c.Q, c.Qpad, c.count, out + off, stream);
        off += (int64_t)7 * c.Q * c.count;
    }
    return hip_status();
}

int hrom_cauchy(hrom_plan plan, double* sigma, double* dsdD, int32_t* status, hipStream_t stream) {
    if (!plan || !sigma || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.stage < 2) return HROM_E_ORDER;
    if (!(p.flags & HROM_OBJECTIVE)) return HROM_E_UNSUPPORTED;
    CauchyArgs ca{p.N, p.polar, p.Palg, p.Cr, sigma, dsdD, status};
    launch_cauchy(ca, stream);
    return hip_status();
}

int hrom_backward(hrom_plan plan, const double* theta, const double* a, const double* gPbar,
                  double* gFbar, double* gtheta, int32_t* status, hipStream_t stream) {
    if (!plan || !theta || !a || !gPbar || !gFbar || !gtheta || !status) return HROM_E_INVALID;
    Plan& p = plan->p;
    if (p.j2) return HROM_E_UNSUPPORTED;   // no adjoint through the plastic history
    if (p.stage < 2) return HROM_E_ORDER;
    const int objective = (p.flags & HROM_OBJECTIVE) ? 1 : 0;
    BwPointArgs bp{p.N, objective, p.polar, p.S, gPbar, p.gr, p.Lam, p.hr, gFbar};
    launch_bw_pullback(bp, stream);
    map_in(p, a, stream);
    for (const auto& c : p.cl) {
        LambdaArgs la{c.m, c.first, c.count, p.N, p.nmac, p.X + (int64_t)p.nmac * c.off_a, p.gr,
                      p.lam + c.off_a, p.conv + c.first};
        launch_lambda(la, stream);
        BackwardArgs ba{};
        ba.m = c.m; ba.Q = c.Q; ba.Qpad = c.Qpad; ba.mixed = mixed(p); ba.objective = objective;
        ba.first = c.first; ba.count = c.count; ba.N = p.N;
        ba.GT = c.GT; ba.Ghat = c.Ghat; ba.Gf = c.Gf; ba.Gb3 = c.Gb3; ba.MP = c.MP; ba.MT = c.MT;
        ba.KS = c.KS;
        ba.w = c.w; ba.phase = c.phase;
        ba.theta = theta; ba.Fr = p.Fr; ba.a = p.at + c.off_a; ba.lam = p.lam + c.off_a;
        ba.gr = p.gr; ba.hr = p.hr; ba.gth = p.gth; ba.rho = p.rho + c.off_a; ba.status = status;
        if (refine(p)) {
            // iterative refinement of the adjoint solve: the residual
            // rho = KaF g_r - Kaa lambda with the accurate (FP32-tangent)
            // operator, corrected with the factor of the low-precision Kaa,
            // until the correction falls below kRefineTol of lambda (per point;
            // at most kRefineSteps steps; HROM_PT_NOREFINE when the last
            // correction is still above kRefineFlagTol of lambda)
            ba.conv = p.conv + c.first;
            for (int step = 0; step < kRefineSteps; step++) {
                ba.with_rho = 1;
                int rc = launch_backward_b(ba, stream);
                if (rc != HROM_OK) return rc;
                RefineArgs ra{c.m, c.first, c.count, p.L + c.ws_L, p.piv + c.off_a, status,
                              p.rho + c.off_a, p.lam + c.off_a, p.conv + c.first, kRefineTol,
                              kRefineFlagTol, step + 1 == kRefineSteps ? 1 : 0};
                launch_refine_lambda(ra, stream);
            }
        }
        // final pass (h_r, dL/dtheta): with refinement also on the FP64
        // operator, so that the low-precision factor only preconditions the
        // solve for lambda
        ba.with_rho = 0;
        if (refine(p)) ba.mixed = 0;
        int rc = launch_backward_b(ba, stream);
        if (rc != HROM_OK) return rc;
    }
    launch_bw_pushforward(bp, stream);
    launch_reduce_theta(p.N, p.gth, p.gth_part, gtheta, stream);
    return hip_status();
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free Newton
// hrom_newton_noalloc: the plan of hrom_plan_create + hrom_newton, with every
// device buffer carved from a file-scope device array instead of hipMalloc.
// The array's device address is looked up once per device (hipGetSymbolAddress
// with that device current) and only that address is handed to kernels.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;   // per device
constexpr int kMaxDevices = 64;
constexpr int kNoallocMaxClusters = 16;

struct NoallocState {
    std::mutex mu;            // serialises host-side use of the device's plan object
    bool ready = false;
    char* ptr = nullptr;      // device address of `scratch` on this device
    hrom_plan_s plan;         // cluster capacity reserved at library load
    NoallocState() { plan.p.cl.reserve(kNoallocMaxClusters); }
};
NoallocState g_noalloc[kMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

extern "C" {

size_t hrom_noalloc_scratch_bytes(void) { return kScratchBytes; }

int hrom_newton_noalloc(const hrom_cluster* clusters, int32_t ncl, int64_t N, int32_t precision,
                        uint32_t flags, const double* theta, const double* Fbar, double* a,
                        double tol, int32_t max_it, double* Pbar, double* Cbar, double* rnorm,
                        int32_t* status, hipStream_t stream) {
    if (!clusters || !theta || !Fbar || !a || !Pbar || !Cbar || !status || max_it < 1 || ncl < 1)
        return HROM_E_INVALID;
    if (ncl > kNoallocMaxClusters || (flags & HROM_J2)) return HROM_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HROM_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return HROM_E_UNSUPPORTED;
    NoallocState& S = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    if (!S.ready) {
        void* addr = nullptr;
        if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || !addr) return HROM_E_HIP;
        S.ptr = static_cast<char*>(addr);
        set_kernel_attributes();
        if (set_basis_attributes() != HROM_OK) return HROM_E_HIP;
        S.ready = true;
    }
    Plan& p = S.plan.p;
    int rc = plan_geometry(p, clusters, ncl, N, precision, flags);
    if (rc != HROM_OK) return rc;
    const size_t bytes = plan_carve(p, nullptr);
    if (bytes > kScratchBytes) return HROM_E_SCRATCH;
    p.device = dev;
    p.arena = S.ptr;
    p.arena_bytes = bytes;
    p.owns_arena = false;
    p.grouped = false;   // one launch per cluster for every step: no device tables
    p.profile = false;
    p.stage = 0;
    plan_carve(p, S.ptr);
    plan_build(p, clusters, stream);
    rc = hip_status();
    if (rc != HROM_OK) return rc;
    return hrom_newton(&S.plan, theta, Fbar, a, tol, max_it, Pbar, Cbar, rnorm, status, stream);
}

}  // extern "C"
