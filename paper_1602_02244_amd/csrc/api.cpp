// C ABI of the FMM library: argument validation, status codes, plan lifetime,
// statistics and exports.  All computation happens in the device kernels of
// plan.hip and eval.hip.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "fmm_internal.h"

namespace fmm {
void build_plan(fmm_plan_s *P, const float *points, hipStream_t s);
void run_eval(fmm_plan_s *Pl, const float *q, float *phi, float *grad, float *hess, int phases, hipStream_t s,
              const float *dip = nullptr);
void run_adjoint_grad(fmm_plan_s *Pl, const float *q, const float *w, const float *g, float *dq, float *dx,
                      hipStream_t s);
void run_adjoint_combine(fmm_plan_s *Pl, const float *w, const float *gphi, const float *q, const float *gpsi, float *dx,
                         hipStream_t s);
}  // namespace fmm

using namespace fmm;

namespace {
thread_local std::string g_err;
std::mutex g_alloc_mu;
fmm_alloc_fn g_alloc = nullptr;
fmm_free_fn g_free = nullptr;
void *g_ctx = nullptr;

fmm_status set_err(fmm_status s, const std::string &m) {
    g_err = m;
    return s;
}

void note_stream(fmm_plan_s *P, hipStream_t s) {
    for (hipStream_t t : P->streams_used)
        if (t == s) return;
    P->streams_used.push_back(s);
}

void destroy_plan(fmm_plan_s *P) {
    if (!P) return;
    const bool log = getenv("FMM_LOG") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    auto stamp = [&](const char *w) {
        if (log)
            fprintf(stderr, "[fmm destroy] %-12s %8.3f ms\n", w,
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    };
    for (hipStream_t st : P->streams_used) (void)hipStreamSynchronize(st);
    if (P->side) (void)hipStreamSynchronize(P->side);
    (void)hipStreamSynchronize(P->mem.stream);
    stamp("synced");
    P->mem.release_all();
    stamp("freed");
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    for (auto &e : P->ev)
        if (e) (void)hipEventDestroy(e);
    stamp("events");
    delete P;
}

// One near-field stream per device, shared by all plans (default priority).
hipStream_t side_stream(int dev) {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : streams)
        if (e.first == dev) return e.second;
    hipStream_t st = nullptr;
    HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams.emplace_back(dev, st);
    return st;
}

template <class F> fmm_status guarded(F &&f) {
    try {
        f();
        return FMM_OK;
    } catch (const Error &e) {
        return set_err(e.status, e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(FMM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(FMM_EDEVICE, "unexpected internal error");
    }
}

void fill_stats(fmm_plan_s *P) {
    fmm_stats &st = P->stats;
    std::memset(&st, 0, sizeof(st));
    st.n = P->n;
    st.p = P->p;
    st.ncrit = P->ncrit;
    st.precision = (int32_t)P->prec;
    st.max_level = P->max_level;
    st.theta = P->theta;
    st.root_exponent = P->k;
    for (int a = 0; a < 3; ++a) st.root_corner[a] = P->x0[a];
    st.ncells = P->ncells;
    st.nleaves = P->nleaves;
    for (int l = 0; l <= P->max_level && l < FMM_MAX_LEVELS; ++l)
        st.cells_per_level[l] = P->level_off[l + 1] - P->level_off[l];
    // leaves per level from a host copy of the child counts
    std::vector<int32_t> nch(P->ncells);
    HIP_CHECK(hipMemcpyAsync(nch.data(), P->c_nchild, 4 * P->ncells, hipMemcpyDeviceToHost, P->mem.stream));
    HIP_CHECK(hipStreamSynchronize(P->mem.stream));
    for (int l = 0; l <= P->max_level && l < FMM_MAX_LEVELS; ++l)
        for (int64_t c = P->level_off[l]; c < P->level_off[l + 1]; ++c) st.leaves_per_level[l] += nch[c] == 0;
    st.m2l_pairs = P->nm2l;
    st.m2l_pairs_same_level = P->nm2l_same;
    st.m2l_keys = P->nkeys;
    st.m2l_keys_same_level = P->nkeys_same;
    st.m2l_targets = P->ntargets;
    st.m2l_tiles = P->ntiles;
    st.m2l_entries = P->nentries;
    st.m2l_work_items = P->nwork;
    st.p2p_pairs = P->np2p;
    st.p2p_interactions = P->p2p_interactions;
    st.ncoef = ncoef(P->p);
    st.ncoef_padded = P->KP;
    double nc = (double)ncoef(P->p);
    st.m2l_flops = 2.0 * nc * nc * (double)P->nm2l;
    st.p2p_flops = 20.0 * (double)P->p2p_interactions;
    st.workspace_bytes = P->mem.bytes;
    st.m2l_tol = P->m2l_tol;
    st.m2l_kept_fraction = P->m2l_kept;
    st.lists = P->lists;
    st.p2p_work_items = P->np2p_items;
    st.p2p_split_pieces = P->np2p_part;
    st.m2l_pool_pairs = P->npool;
    st.m2l_slots = P->nslots;
    st.m2l_slot_tiles = P->nslot_tiles;
    st.svd_tol = P->svd_tol;
    st.m2l_svd_rank_mean = P->svd_rank_mean;
}
}  // namespace

extern "C" {

const char *fmm_last_error(void) { return g_err.c_str(); }

fmm_status fmm_set_allocator(fmm_alloc_fn alloc, fmm_free_fn release, void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) return set_err(FMM_EINVAL, "allocator and release must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = alloc;
    g_free = release;
    g_ctx = ctx;
    return FMM_OK;
}

fmm_status fmm_plan(const float *points, int64_t n, int ncrit, int p, float theta, fmm_precision prec, void *stream,
                    fmm_plan_t *out) {
    return fmm_plan_ex(points, n, ncrit, p, theta, prec, 0.0, FMM_LISTS_DUAL, stream, out);
}

// A plan over `points` [n][3], or (targets != NULL) over the union of n sources and nt
// targets, sources first.
static fmm_status plan_create(const float *points, int64_t n, const float *targets, int64_t nt, int ncrit, int p,
                              float theta, fmm_precision prec, double m2l_tol, int lists, void *stream,
                              fmm_plan_t *out, double svd_tol = 0.0) {
    if (!out) return set_err(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!points) return set_err(FMM_EINVAL, "points is NULL");
    if (n < 1) return set_err(FMM_EINVAL, "n must be >= 1");
    if (targets && nt < 1) return set_err(FMM_EINVAL, "nt must be >= 1");
    if (targets && n >= (int64_t(1) << 31) - 1 - nt) return set_err(FMM_EUNSUPPORTED, "ns + nt must be below 2^31 - 1");
    const int64_t nsrc = n;
    if (targets) n += nt;
    else nt = 0;
    if (n >= (int64_t(1) << 31) - 1) return set_err(FMM_EUNSUPPORTED, "n must be below 2^31 - 1");
    if (ncrit < 1) return set_err(FMM_EINVAL, "ncrit must be >= 1");
    if (p < 0 || p > kMaxP) return set_err(FMM_EINVAL, "p must be in [0, 16]");
    if (!std::isfinite(theta) || !(theta > 0.f) || !(3.0 * (double)theta * (double)theta < 1.0))
        return set_err(FMM_EINVAL, "theta must be in (0, 1/sqrt(3))");
    if (prec != FMM_PREC_FP32 && prec != FMM_PREC_MIXED) return set_err(FMM_EINVAL, "unknown precision");
    if (!std::isfinite(m2l_tol) || m2l_tol < 0.0) return set_err(FMM_EINVAL, "m2l_tol must be finite and >= 0");
    if (m2l_tol > 0.0 && prec != FMM_PREC_FP32)
        return set_err(FMM_EINVAL, "a variable-order M2L (m2l_tol > 0) needs FMM_PREC_FP32");
    if (lists != FMM_LISTS_DUAL && lists != FMM_LISTS_LEVEL_SKIP) return set_err(FMM_EINVAL, "unknown lists value");
    if (!std::isfinite(svd_tol) || svd_tol < 0.0 || svd_tol >= 1.0)
        return set_err(FMM_EINVAL, "svd_tol must be in [0, 1)");
    if (svd_tol > 0.0 && prec != FMM_PREC_FP32)
        return set_err(FMM_EINVAL, "an SVD-compressed M2L (svd_tol > 0) needs FMM_PREC_FP32");
    fmm_plan_s *P = new (std::nothrow) fmm_plan_s();
    if (!P) return set_err(FMM_ENOMEM, "host allocation failed");
    P->n = n;
    P->nsrc = nsrc;
    P->ntgt = nt;
    P->ncrit = ncrit;
    P->p = p;
    P->theta = theta;
    P->prec = prec;
    P->m2l_tol = m2l_tol;
    P->svd_tol = svd_tol;
    P->lists = lists;
    P->KP = ncoef_pad(p);
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        P->mem.alloc = g_alloc;
        P->mem.release = g_free;
        P->mem.ctx = g_ctx;
    }
    hipStream_t s = (hipStream_t)stream;
    P->mem.stream = s;
    note_stream(P, s);
    fmm_status st = guarded([&] {
        HIP_CHECK(hipGetDevice(&P->device));
        P->side = side_stream(P->device);
        HIP_CHECK(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
        if (nt > 0) {   // the union point set, sources first
            float *uni = P->mem.get_n<float>(3 * n);
            HIP_CHECK(hipMemcpyAsync(uni, points, sizeof(float) * 3 * nsrc, hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipMemcpyAsync(uni + 3 * nsrc, targets, sizeof(float) * 3 * nt, hipMemcpyDeviceToDevice, s));
            build_plan(P, uni, s);   // ends with a synchronisation
            P->mem.put(uni);
        } else {
            build_plan(P, points, s);
        }
        fill_stats(P);
    });
    if (st != FMM_OK) {
        destroy_plan(P);
        return st;
    }
    *out = P;
    return FMM_OK;
}

fmm_status fmm_plan_ex(const float *points, int64_t n, int ncrit, int p, float theta, fmm_precision prec,
                       double m2l_tol, int lists, void *stream, fmm_plan_t *out) {
    return plan_create(points, n, nullptr, 0, ncrit, p, theta, prec, m2l_tol, lists, stream, out);
}

fmm_status fmm_plan_svd(const float *points, int64_t n, int ncrit, int p, float theta, double svd_tol, void *stream,
                        fmm_plan_t *out) {
    return plan_create(points, n, nullptr, 0, ncrit, p, theta, FMM_PREC_FP32, 0.0, FMM_LISTS_DUAL, stream, out,
                       svd_tol);
}

fmm_status fmm_plan_targets(const float *sources, int64_t ns, const float *targets, int64_t nt, int ncrit, int p,
                            float theta, fmm_precision prec, void *stream, fmm_plan_t *out) {
    if (!targets) {
        if (out) *out = nullptr;
        return set_err(FMM_EINVAL, "targets is NULL");
    }
    return plan_create(sources, ns, targets, nt, ncrit, p, theta, prec, 0.0, FMM_LISTS_DUAL, stream, out);
}

fmm_status fmm_eval_ex(fmm_plan_t plan, const float *charges, float *potential, float *gradient, int phases,
                       void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (!charges) return set_err(FMM_EINVAL, "charges is NULL");
    if (!potential && !gradient) return set_err(FMM_EINVAL, "potential and gradient are both NULL");
    if (phases < 1 || phases > 3) return set_err(FMM_EINVAL, "phases must be a non-empty subset of FMM_NEAR | FMM_FAR");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_eval_targets");
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        note_stream(plan, s);
        run_eval(plan, charges, potential, gradient, nullptr, phases, s);
    });
}

fmm_status fmm_eval(fmm_plan_t plan, const float *charges, float *potential, float *gradient, void *stream) {
    return fmm_eval_ex(plan, charges, potential, gradient, FMM_ALL, stream);
}

// Scratch of the adjoint evaluations (allocated on first use, on the calling stream)
static void adjoint_scratch(fmm_plan_s *P, hipStream_t s) {
    if (P->tmp_phi) return;
    hipStream_t keep = P->mem.stream;
    P->mem.stream = s;
    P->tmp_phi = P->mem.get_n<float>(P->n);
    P->tmp_grad = P->mem.get_n<float>(3 * P->n);
    P->tmp_gfwd = P->mem.get_n<float>(3 * P->n);
    P->mem.stream = keep;
}

fmm_status fmm_adjoint(fmm_plan_t plan, const float *charges, const float *gradient_fwd, const float *dL_dphi,
                       float *dL_dq, float *dL_dx, void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (!dL_dphi) return set_err(FMM_EINVAL, "dL_dphi is NULL");
    if (dL_dx && !charges) return set_err(FMM_EINVAL, "charges is NULL");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_adjoint_targets");
    if (!dL_dq && !dL_dx) return FMM_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        fmm_plan_s *P = plan;
        note_stream(P, s);
        adjoint_scratch(P, s);
        // psi = A w and grad psi: the same FMM with charges w (A is symmetric)
        run_eval(P, dL_dphi, dL_dq ? dL_dq : P->tmp_phi, dL_dx ? P->tmp_grad : nullptr, nullptr, FMM_ALL, s);
        if (dL_dx) {
            const float *gphi = gradient_fwd;
            if (!gphi) {
                run_eval(P, charges, nullptr, P->tmp_gfwd, nullptr, FMM_ALL, s);
                gphi = P->tmp_gfwd;
            }
            run_adjoint_combine(P, dL_dphi, gphi, charges, P->tmp_grad, dL_dx, s);
        }
    });
}

// ---- the adjoint without allocation: scratch in a static device array
}  // extern "C"

namespace {
constexpr int64_t kNoallocFloats = 7 * FMM_NOALLOC_MAX_N;   // psi [n], grad psi [n][3], grad phi [n][3]
__device__ __align__(256) float scratch[kNoallocFloats];
std::mutex g_scratch_mu;
std::vector<std::pair<int, float *>> g_scratch_ptr;   // device -> address of `scratch` there

// Address of `scratch` on device `dev` (the current device), looked up once per device.
// Host code never uses the array's own name as an address.
float *noalloc_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    for (auto &e : g_scratch_ptr)
        if (e.first == dev) return e.second;
    void *ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(FMM_EDEVICE, "hipGetSymbolAddress returned NULL for the static scratch");
    g_scratch_ptr.emplace_back(dev, static_cast<float *>(ptr));
    return static_cast<float *>(ptr);
}
}  // namespace

extern "C" {

fmm_status fmm_adjoint_noalloc(fmm_plan_t plan, const float *charges, const float *gradient_fwd,
                               const float *dL_dphi, float *dL_dq, float *dL_dx, void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (!dL_dphi) return set_err(FMM_EINVAL, "dL_dphi is NULL");
    if (dL_dx && !charges) return set_err(FMM_EINVAL, "charges is NULL");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_adjoint_targets");
    if (plan->n > FMM_NOALLOC_MAX_N)
        return set_err(FMM_EINVAL, "fmm_adjoint_noalloc takes plans of at most 2^20 points (its static scratch); "
                                   "this plan has " + std::to_string(plan->n));
    if (!dL_dq && !dL_dx) return FMM_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        fmm_plan_s *P = plan;
        int dev = -1;
        HIP_CHECK(hipGetDevice(&dev));
        if (dev != P->device) fail(FMM_EINVAL, "the current device is not the plan's device");
        float *sc = noalloc_scratch(dev);
        const int64_t n = P->n;
        float *psi = sc, *gpsi = sc + n, *gfwd = sc + 4 * n;
        note_stream(P, s);
        run_eval(P, dL_dphi, dL_dq ? dL_dq : psi, dL_dx ? gpsi : nullptr, nullptr, FMM_ALL, s);
        if (dL_dx) {
            const float *gphi = gradient_fwd;
            if (!gphi) {
                run_eval(P, charges, nullptr, gfwd, nullptr, FMM_ALL, s);
                gphi = gfwd;
            }
            run_adjoint_combine(P, dL_dphi, gphi, charges, gpsi, dL_dx, s);
        }
    });
}

fmm_status fmm_eval_hessian(fmm_plan_t plan, const float *charges, float *potential, float *gradient, float *hessian,
                            void *stream) {
    if (!plan || !charges || !hessian) return set_err(FMM_EINVAL, "NULL argument");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_eval_targets");
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        note_stream(plan, s);
        run_eval(plan, charges, potential, gradient, hessian, FMM_ALL, s);
    });
}

fmm_status fmm_eval_dipoles(fmm_plan_t plan, const float *charges, const float *dipoles, float *potential,
                            float *gradient, void *stream) {
    if (!plan || !charges || !dipoles) return set_err(FMM_EINVAL, "NULL argument");
    if (!potential && !gradient) return set_err(FMM_EINVAL, "potential and gradient are both NULL");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_eval_targets");
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        note_stream(plan, s);
        run_eval(plan, charges, potential, gradient, nullptr, FMM_ALL, s, dipoles);
    });
}

fmm_status fmm_adjoint_ex(fmm_plan_t plan, const float *charges, const float *dL_dphi, const float *dL_dgrad,
                          float *dL_dq, float *dL_dx, void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (!charges || !dL_dphi || !dL_dgrad) return set_err(FMM_EINVAL, "NULL argument");
    if (plan->ntgt > 0) return set_err(FMM_EINVAL, "a plan with a separate target set takes fmm_adjoint_targets");
    if (!dL_dq && !dL_dx) return FMM_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        fmm_plan_s *P = plan;
        note_stream(P, s);
        adjoint_scratch(P, s);
        run_adjoint_grad(P, charges, dL_dphi, dL_dgrad, dL_dq, dL_dx, s);
    });
}

// ------------------------------------------------------------ separate target set
// The union problem: charges [q; 0], loss weights [0; w] (and [0; g]); its evaluation and
// adjoint restricted to the targets / sources are those of the two-set problem.
namespace {
struct TargetScratch {   // union-sized views into the plan's scratch (allocated on first use)
    float *q, *w, *g, *phi, *grad, *dq, *dx, *gpsi;
};
TargetScratch target_scratch(fmm_plan_s *P, hipStream_t s) {
    const int64_t n = P->n;
    if (!P->tmp_u) {
        hipStream_t keep = P->mem.stream;
        P->mem.stream = s;
        P->tmp_u = P->mem.get_n<float>(5 * n);   // q, w, g (or the forward gradient)
        P->tmp_o = P->mem.get_n<float>(11 * n);  // phi, grad, dq, dx, grad psi
        P->mem.stream = keep;
    }
    return TargetScratch{P->tmp_u, P->tmp_u + n, P->tmp_u + 2 * n, P->tmp_o, P->tmp_o + n, P->tmp_o + 4 * n,
                         P->tmp_o + 5 * n, P->tmp_o + 8 * n};
}
// dst[0, n*w) = src placed at items [off, off + cnt), zero elsewhere
void embed(float *dst, int64_t n, int w, const float *src, int64_t off, int64_t cnt, hipStream_t s) {
    if (off > 0) fill_f32(dst, 0.f, off * w, s);
    if (off + cnt < n) fill_f32(dst + (off + cnt) * w, 0.f, (n - off - cnt) * w, s);
    HIP_CHECK(hipMemcpyAsync(dst + off * w, src, sizeof(float) * cnt * w, hipMemcpyDeviceToDevice, s));
}
void extract(float *dst, const float *src, int w, int64_t off, int64_t cnt, hipStream_t s) {
    if (dst) HIP_CHECK(hipMemcpyAsync(dst, src + off * w, sizeof(float) * cnt * w, hipMemcpyDeviceToDevice, s));
}
}  // namespace

fmm_status fmm_eval_targets(fmm_plan_t plan, const float *charges, float *potential, float *gradient, void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (plan->ntgt == 0) return set_err(FMM_EINVAL, "the plan has no separate target set (use fmm_eval)");
    if (!charges) return set_err(FMM_EINVAL, "charges is NULL");
    if (!potential && !gradient) return set_err(FMM_EINVAL, "potential and gradient are both NULL");
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        fmm_plan_s *P = plan;
        note_stream(P, s);
        const TargetScratch t = target_scratch(P, s);
        embed(t.q, P->n, 1, charges, 0, P->nsrc, s);
        run_eval(P, t.q, potential ? t.phi : nullptr, gradient ? t.grad : nullptr, nullptr, FMM_ALL, s);
        extract(potential, t.phi, 1, P->nsrc, P->ntgt, s);
        extract(gradient, t.grad, 3, P->nsrc, P->ntgt, s);
    });
}

fmm_status fmm_adjoint_targets(fmm_plan_t plan, const float *charges, const float *gradient_fwd, const float *dL_dphi,
                               const float *dL_dgrad, float *dL_dq, float *dL_dx_src, float *dL_dx_tgt,
                               void *stream) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    if (plan->ntgt == 0) return set_err(FMM_EINVAL, "the plan has no separate target set (use fmm_adjoint)");
    if (!charges || !dL_dphi) return set_err(FMM_EINVAL, "NULL argument");
    if (!dL_dq && !dL_dx_src && !dL_dx_tgt) return FMM_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        fmm_plan_s *P = plan;
        note_stream(P, s);
        const int64_t n = P->n, ns = P->nsrc, nt = P->ntgt;
        const TargetScratch t = target_scratch(P, s);
        const bool want_dx = dL_dx_src || dL_dx_tgt;
        embed(t.q, n, 1, charges, 0, ns, s);
        embed(t.w, n, 1, dL_dphi, ns, nt, s);
        if (dL_dgrad) {   // losses through grad phi: the Hessian FMM (five evaluations)
            adjoint_scratch(P, s);
            embed(t.g, n, 3, dL_dgrad, ns, nt, s);
            run_adjoint_grad(P, t.q, t.w, t.g, dL_dq ? t.dq : nullptr, want_dx ? t.dx : nullptr, s);
        } else {
            // psi = A w_u and grad psi; dL/dx_u = w_u grad phi + q_u grad psi
            run_eval(P, t.w, t.dq, want_dx ? t.gpsi : nullptr, nullptr, FMM_ALL, s);
            if (want_dx) {
                if (gradient_fwd) embed(t.g, n, 3, gradient_fwd, ns, nt, s);   // zero at sources: w is 0 there
                else run_eval(P, t.q, nullptr, t.g, nullptr, FMM_ALL, s);
                run_adjoint_combine(P, t.w, t.g, t.q, t.gpsi, t.dx, s);
            }
        }
        extract(dL_dq, t.dq, 1, 0, ns, s);
        extract(dL_dx_src, t.dx, 3, 0, ns, s);
        extract(dL_dx_tgt, t.dx, 3, ns, nt, s);
    });
}

fmm_status fmm_plan_stats(fmm_plan_t plan, struct fmm_stats *out) {
    if (!plan || !out) return set_err(FMM_EINVAL, "NULL argument");
    *out = plan->stats;
    out->workspace_bytes = plan->mem.bytes;
    return FMM_OK;
}

fmm_status fmm_plan_export(fmm_plan_t plan, int32_t *level, uint64_t *prefix, int64_t *start, int64_t *count,
                           int32_t *leaf, int64_t *order, int64_t *m2l, int64_t *p2p) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    fmm_plan_s *P = plan;
    hipStream_t s = P->mem.stream;
    return guarded([&] {
        const int64_t nc = P->ncells;
        std::vector<int32_t> tmp;
        auto i32 = [&](const int32_t *dev, int64_t nn) {
            tmp.resize(nn);
            HIP_CHECK(hipMemcpyAsync(tmp.data(), dev, 4 * nn, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
        };
        if (level) {
            i32(P->c_level, nc);
            std::memcpy(level, tmp.data(), 4 * nc);
        }
        if (prefix) {
            HIP_CHECK(hipMemcpyAsync(prefix, P->c_prefix_dev, 8 * nc, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        if (start) { i32(P->c_start, nc); for (int64_t c = 0; c < nc; ++c) start[c] = tmp[c]; }
        if (count) { i32(P->c_count, nc); for (int64_t c = 0; c < nc; ++c) count[c] = tmp[c]; }
        if (leaf) { i32(P->c_nchild, nc); for (int64_t c = 0; c < nc; ++c) leaf[c] = tmp[c] == 0; }
        if (order) { i32(P->perm, P->n); for (int64_t i = 0; i < P->n; ++i) order[i] = tmp[i]; }
        auto pairs = [&](const int2 *dev, int64_t np, int64_t *outp) {
            std::vector<int2> h(np);
            if (np > 0) {
                HIP_CHECK(hipMemcpyAsync(h.data(), dev, sizeof(int2) * np, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
            }
            for (int64_t i = 0; i < np; ++i) { outp[2 * i] = h[i].x; outp[2 * i + 1] = h[i].y; }
        };
        if (m2l) pairs(P->m2l_pairs, P->nm2l, m2l);
        if (p2p) pairs(P->p2p_pairs, P->np2p, p2p);
    });
}

fmm_status fmm_plan_set_timing(fmm_plan_t plan, int enable) {
    if (!plan) return set_err(FMM_EINVAL, "plan is NULL");
    return guarded([&] {
        if (enable && !plan->ev[0])
            for (auto &e : plan->ev) HIP_CHECK(hipEventCreate(&e));
        plan->timing = enable != 0;
        plan->ev_valid = false;
    });
}

fmm_status fmm_plan_phase_times(fmm_plan_t plan, float *ms) {
    if (!plan || !ms) return set_err(FMM_EINVAL, "NULL argument");
    if (!plan->ev_valid) return set_err(FMM_EINVAL, "no timed evaluation recorded (enable timing first)");
    return guarded([&] {
        for (int ph = 0; ph < FMM_NUM_PHASES; ++ph) {
            HIP_CHECK(hipEventSynchronize(plan->ev[2 * ph + 1]));
            HIP_CHECK(hipEventElapsedTime(&ms[ph], plan->ev[2 * ph], plan->ev[2 * ph + 1]));
        }
    });
}

void fmm_plan_destroy(fmm_plan_t plan) { destroy_plan(plan); }

}  // extern "C"
