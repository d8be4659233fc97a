// prs_api.cpp -- host side of the C ABI declared in include/prs.h: argument
// validation, run contexts, the FP64 coefficient schedule of Eqs. (4)-(6)
// and the Eq. (9) exponent fit.  Every step of the evolution runs in the
// kernels of prs_device.h (float32 and float64 instantiations).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstddef>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "prs.h"
#include "prs_internal.h"

using namespace prs;

namespace {

thread_local char g_err[512] = "";

prs_status fail(prs_status s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

prs_status hip_fail(hipError_t e, const char* what)
{
    return fail(PRS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kRecCap = 1024;   // device records buffered before a flush
constexpr int64_t kMinRows = 8;     // smallest marching tile the workspace allows

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double v0_of(const prs_params& p)
{
    return std::isinf(p.W0) ? 0.0 : M_PI * M_PI / (2.0 * p.W0 * p.W0);
}

int64_t sites_of(const prs_params& p)
{
    return p.n[0] * p.n[1] * (p.ndim == 3 ? p.n[2] : 1);
}

// Bytes of one field value.
size_t esize_of(const prs_params& p) { return p.precision == PRS_F64 ? 8 : 4; }

size_t field_bytes(const prs_params& p) { return (size_t)sites_of(p) * esize_of(p); }

template <typename T>
T* byte_offset(void* base, size_t off)
{
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

prs_status validate(const prs_params* p)
{
    if (!p) return fail(PRS_EINVAL, "params is NULL");
    if (p->ndim != 2 && p->ndim != 3) return fail(PRS_EINVAL, "ndim must be 2 or 3 (got %d)", p->ndim);
    for (int d = 0; d < p->ndim; ++d)
        if (p->n[d] < 1) return fail(PRS_EINVAL, "lattice side n[%d] = %lld must be >= 1", d, (long long)p->n[d]);
    const double lim = 1.0 * (1ll << 40);
    double sites = 1.0;
    for (int d = 0; d < p->ndim; ++d) sites *= (double)p->n[d];
    if (sites > lim) return fail(PRS_EINVAL, "lattice too large (%.3g sites)", sites);
    if ((double)p->n[0] * (double)(p->ndim == 3 ? p->n[1] : 1) > 2147483647.0)
        return fail(PRS_EINVAL, "a lattice plane (nx in 2D, nx*ny in 3D) must hold fewer than 2^31 sites");
    if (!(p->dx > 0) || !std::isfinite(p->dx)) return fail(PRS_EINVAL, "dx must be finite and > 0");
    if (!(p->deta > 0) || !std::isfinite(p->deta)) return fail(PRS_EINVAL, "deta must be finite and > 0");
    if (!(p->eta0 > 0) || !std::isfinite(p->eta0)) return fail(PRS_EINVAL, "eta0 must be finite and > 0");
    if (!(p->alpha >= 0) || !std::isfinite(p->alpha)) return fail(PRS_EINVAL, "alpha must be finite and >= 0");
    if (!(p->m >= 0) || !std::isfinite(p->m)) return fail(PRS_EINVAL, "m must be finite and >= 0");
    if (!(p->W0 > 0)) return fail(PRS_EINVAL, "W0 must be > 0");
    if (!(p->phi0 > 0) || !std::isfinite(p->phi0)) return fail(PRS_EINVAL, "phi0 must be finite and > 0");
    if (p->diag_every < 0) return fail(PRS_EINVAL, "diag_every must be >= 0");
    if (p->precision != PRS_F32 && p->precision != PRS_F64)
        return fail(PRS_EINVAL, "precision must be PRS_F32 or PRS_F64 (got %d)", p->precision);
    if (p->reserved != 0) return fail(PRS_EINVAL, "reserved must be 0");
    if (!std::isfinite(p->beta)) return fail(PRS_EINVAL, "beta must be finite");
    const double V0 = v0_of(*p);
    const double w2 = 4.0 * p->ndim / (p->dx * p->dx) + 8.0 * V0 / (p->phi0 * p->phi0);
    if (!(p->deta * std::sqrt(w2) < 2.0))
        return fail(PRS_EINVAL, "unstable step: deta*sqrt(4D/dx^2 + 8 V0/phi0^2) = %g must be < 2",
                    p->deta * std::sqrt(w2));
    const double d0 = 0.5 * p->alpha * (p->deta / p->eta0) * p->m;
    if (!(d0 < 1.0)) return fail(PRS_EINVAL, "first damping factor delta_0 = %g must be < 1", d0);
    return PRS_OK;
}

Tiling default_tiling(const Geometry& g)
{
    Tiling t;
    if (g.nx % 4 == 0 && g.nx >= 256) t.vec = 4;
    else if (g.nx % 2 == 0 && g.nx >= 128) t.vec = 2;
    else if (g.nx % 4 == 0) t.vec = 4;
    else if (g.nx % 2 == 0) t.vec = 2;
    else t.vec = 1;
    if (g.f64 && t.vec == 4) t.vec = 2;   // 16 bytes per lane at most
    t.ty = g.ndim == 3 ? 2 : 1;
    t.rows = g.ndim == 3 ? 32 : 16;
    return t;
}

int64_t partial_capacity(const Geometry& g)
{
    Tiling t{1, (int)kMinRows, 1};
    int64_t n = tile_counts(g, t).ntiles;
    if (g.ndim == 2) n = std::max<int64_t>(n, tb_tiles(g, t, kMaxPassSteps));
    else {
        n = std::max<int64_t>(n, tb_tiles(g, t, 3));    // 3D: 4 owned rows, T <= 3
        // the LDS pass: one partial per wave, 2 rows per wave, T <= 4
        n = std::max<int64_t>(n, tb_tiles(g, Tiling{1, (int)kMinRows, 8}, 4));
    }
    return n;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Steps of each pass for nsteps steps from n0 with up to T steps per pass:
// no pass has a recorded state (n % K == 0, K > 0) strictly inside it, every
// multi-step pass has a length with a kernel (the longest that fits), and
// the number of multi-step passes is even (each flips the phi_dot buffer, so
// phi_dot ends where it started).
std::vector<uint8_t> plan_passes(const Geometry& g, const Tiling& t, int64_t cap, int64_t n0, int64_t nsteps, int T,
                                 int64_t K)
{
    // a length needs a kernel for the tiling and at most `cap` wave tiles
    // (the partial buffers hold that many)
    auto ok = [&](int L) { return tb_pass_supported(g, t, L) && tb_tiles(g, t, L) <= cap; };
    std::vector<uint8_t> plan;
    int64_t nmulti = 0;
    for (int64_t n = n0; n < n0 + nsteps;) {
        int64_t L = std::min<int64_t>(T, n0 + nsteps - n);
        if (K > 0) L = std::min<int64_t>(L, (n / K + 1) * K - n);
        while (L > 1 && !ok((int)L)) --L;
        plan.push_back((uint8_t)L);
        nmulti += L > 1 ? 1 : 0;
        n += L;
    }
    if (nmulti % 2 == 1) {
        // one flip too many: split the last multi-step pass, into two halves
        // when both are multi-step lengths (4 -> 2+2, 6 -> 3+3, 8 -> 4+4),
        // otherwise into single steps
        for (size_t i = plan.size(); i-- > 0;)
            if (plan[i] > 1) {
                const int L = plan[i];
                const int a = L / 2, b = L - a;
                plan.erase(plan.begin() + (std::ptrdiff_t)i);
                if (a > 1 && ok(a) && ok(b)) {
                    plan.insert(plan.begin() + (std::ptrdiff_t)i, (uint8_t)b);
                    plan.insert(plan.begin() + (std::ptrdiff_t)i, (uint8_t)a);
                } else {
                    plan.insert(plan.begin() + (std::ptrdiff_t)i, (size_t)L, (uint8_t)1);
                }
                break;
            }
    }
    return plan;
}

}  // namespace

struct prs_ctx {
    prs_params p;
    Geometry geo;
    Tiling til;
    double V0;
    void* phi[2];      // float32 or float64 fields, as p.precision says
    int cur;
    void* pi;
    WavePartial* partials;
    int64_t partial_cap;
    prs_stats* drec;
    prs_stats* hrec;   // pinned staging buffer
    void* pi_alt;      // second phi_dot buffer (workspace) for multi-step passes
    Tiling adj_til;    // tiling of the reverse-sweep kernel
    int32_t adj_tblock;   // steps per reverse pass
    int32_t adj_scheme;   // PRS_ADJ_STORED or PRS_ADJ_FUSED
    Tiling rec_til;    // tiling and steps per pass of the adjoint's recomputation
    int32_t rec_tblock;   // (0: those of the forward)
    int32_t tblock;    // steps per pass (1: single steps)
    hipStream_t stream;
    int64_t step;
    // adjoint bookkeeping between prs_adjoint_forward and _backward
    bool adj_ready;
    int64_t adj_n0, adj_nsteps;
    int32_t adj_K;
    void* adj_work;
    size_t adj_bytes;
    double* adj_host;   // pinned: loss, G
    // second stream and events of the backward sweep (created on first use):
    // the recomputation of the next-older segment overlaps the reverse sweep
    hipStream_t adj_aux;
    hipEvent_t adj_ev[5];   // 0: forward done, 1-2: segment recomputed, 3-4: segment swept
    // launch timing (prs_set_launch_timing): event pairs bracketing each run
    // of consecutive launches of the pass kernel, with the launches per run
    bool lt_on;
    std::vector<hipEvent_t> lt_ev;
    std::vector<int64_t> lt_count;
    double lt_ms;
    int64_t lt_launches;
};

namespace {

// a(eta_n)^beta with a(eta) = (eta/eta0)^m: the scale-factor power of the
// force of Eq. (2) at step n; exactly 1 for the PRS choice beta = 0.
double force_scale(const prs_params& p, int64_t n)
{
    if (p.beta == 0.0) return 1.0;
    return std::pow(std::pow((p.eta0 + (double)n * p.deta) / p.eta0, p.m), p.beta);
}

StepCoef64 coef_for(const prs_ctx* c, int64_t n)
{
    const prs_params& p = c->p;
    const double eta = p.eta0 + (double)n * p.deta;
    const double delta = 0.5 * p.alpha * (p.deta / eta) * p.m;   // Eq. (6)
    StepCoef64 k;
    k.a = (1.0 - delta) / (1.0 + delta);
    k.b = p.deta / (1.0 + delta);
    k.deta = p.deta;
    k.F = 4.0 * c->V0 / (p.phi0 * p.phi0) * force_scale(p, n);
    k.kc = 1.0 / (p.phi0 * p.phi0);
    k.inv_dx2 = 1.0 / (p.dx * p.dx);
    return k;
}

// With beta != 0 the force grows (beta m > 0) or shrinks with eta; the
// linearised stability bound of prs_init, deta sqrt(4D/dx^2 + V''(phi0)
// a^beta) < 2 with V''(phi0) = 8 V0/phi0^2, is checked at the largest force a
// call reaches (its first or its last step).
prs_status check_stable_until(const prs_params& p, double V0, int64_t n_last)
{
    if (p.beta == 0.0) return PRS_OK;
    const double A = std::max(force_scale(p, n_last), force_scale(p, 0));
    const double w2 = 4.0 * p.ndim / (p.dx * p.dx) + 8.0 * V0 / (p.phi0 * p.phi0) * A;
    if (!(p.deta * std::sqrt(w2) < 2.0))
        return fail(PRS_EINVAL, "unstable step %lld with beta = %g: deta*sqrt(4D/dx^2 + 8 V0 a^beta/phi0^2) = %g "
                    "must be < 2", (long long)n_last, p.beta, p.deta * std::sqrt(w2));
    return PRS_OK;
}

// The float32 rounding a float32 launch applies (batched descriptors hold
// float32 coefficients).
StepCoef f32_of(const StepCoef64& k)
{
    return StepCoef{(float)k.a, (float)k.b, (float)k.deta, (float)k.F, (float)k.kc, (float)k.inv_dx2};
}

// Diagnostics of state n: the wall's potential energy in Eq. (8) is
// a(eta_n)^beta V (a static wall has (1/2) phi'^2 = a^beta V).
DiagCoef diag_coef(const prs_ctx* c, int64_t n)
{
    DiagCoef d;
    d.V0 = c->V0 * force_scale(c->p, n);
    d.kc = 1.0 / (c->p.phi0 * c->p.phi0);
    return d;
}

double area_scale(const prs_params& p)
{
    // Eq. (7): Delta A = dx^(D-1) per link over the volume sites * dx^D
    return std::pow(p.dx, p.ndim - 1) / ((double)sites_of(p) * std::pow(p.dx, p.ndim));
}

prs_status flush(prs_ctx* c, int64_t count, prs_stats* dst)
{
    if (count == 0) return PRS_OK;
    HIP_TRY(hipMemcpyAsync(c->hrec, c->drec, (size_t)count * sizeof(prs_stats),
                           hipMemcpyDeviceToHost, c->stream),
            "record copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    std::memcpy(dst, c->hrec, (size_t)count * sizeof(prs_stats));
    return PRS_OK;
}

}  // namespace

extern "C" {

size_t prs_workspace_bytes(const prs_params* p)
{
    if (validate(p) != PRS_OK) return 0;
    const Geometry g = geometry_of(*p);
    size_t b = align_up((size_t)partial_capacity(g) * sizeof(WavePartial)) +
               align_up((size_t)kRecCap * sizeof(prs_stats));
    b += align_up(field_bytes(*p));   // second phi_dot for multi-step passes
    return b;
}

prs_status prs_init(const prs_params* p, void* phi_a, void* phi_b, void* dphi, void* workspace,
                    size_t ws_bytes, void* hip_stream, prs_ctx** out)
{
    if (!out) return fail(PRS_EINVAL, "out is NULL");
    *out = nullptr;
    prs_status st = validate(p);
    if (st != PRS_OK) return st;
    if (!phi_a || !phi_b || !dphi || !workspace) return fail(PRS_EINVAL, "NULL buffer");
    if (!aligned16(phi_a) || !aligned16(phi_b) || !aligned16(dphi))
        return fail(PRS_EINVAL, "field buffers must be 16-byte aligned");
    if (((uintptr_t)workspace % kAlign) != 0) return fail(PRS_EINVAL, "workspace must be 256-byte aligned");
    if (phi_a == phi_b || phi_a == dphi || phi_b == dphi)
        return fail(PRS_EINVAL, "phi_a, phi_b and dphi must be distinct buffers");
    const size_t need = prs_workspace_bytes(p);
    if (ws_bytes < need)
        return fail(PRS_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);

    prs_ctx* c = new (std::nothrow) prs_ctx();
    if (!c) return fail(PRS_ENOMEM, "host allocation failed");
    c->p = *p;
    c->geo = geometry_of(*p);
    c->til = default_tiling(c->geo);
    c->V0 = v0_of(*p);
    c->phi[0] = phi_a;
    c->phi[1] = phi_b;
    c->cur = 0;
    c->pi = dphi;
    c->partial_cap = partial_capacity(c->geo);
    c->partials = static_cast<WavePartial*>(workspace);
    c->drec = reinterpret_cast<prs_stats*>(
        static_cast<char*>(workspace) + align_up((size_t)c->partial_cap * sizeof(WavePartial)));
    c->pi_alt = nullptr;
    c->adj_til = c->til;
    c->adj_tblock = p->ndim == 2 ? 4 : 1;
    c->adj_scheme = p->ndim == 2 ? PRS_ADJ_FUSED : PRS_ADJ_STORED;
    c->pi_alt = reinterpret_cast<char*>(c->drec) + align_up((size_t)kRecCap * sizeof(prs_stats));
    c->tblock = p->ndim == 2 ? 2 : 1;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->step = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->hrec), (size_t)kRecCap * sizeof(prs_stats),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "pinned record buffer");
    }
    *out = c;
    return PRS_OK;
}

int64_t prs_records_in(const prs_params* p, int64_t n0, int64_t nsteps)
{
    if (!p || p->diag_every <= 0 || nsteps <= 0 || n0 < 0) return 0;
    const int64_t K = p->diag_every;
    const int64_t first = (n0 + K - 1) / K * K;
    const int64_t last = n0 + nsteps - 1;
    return last < first ? 0 : (last - first) / K + 1;
}

prs_status prs_step_n(prs_ctx* c, int64_t nsteps, prs_stats* series, int64_t cap, int64_t* n_written)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (n_written) *n_written = 0;
    if (nsteps < 0) return fail(PRS_EINVAL, "nsteps must be >= 0");
    const bool want = series != nullptr && c->p.diag_every > 0;
    const int64_t need = want ? prs_records_in(&c->p, c->step, nsteps) : 0;
    if (want && cap < need)
        return fail(PRS_EINVAL, "series capacity %lld < %lld records", (long long)cap, (long long)need);
    if (nsteps > 0) {
        prs_status st = check_stable_until(c->p, c->V0, c->step + nsteps - 1);
        if (st != PRS_OK) return st;
    }
    const double ascale = area_scale(c->p);
    const TileCounts tc = tile_counts(c->geo, c->til);
    const int64_t K = c->p.diag_every;

    const int T = tb_supported(c->geo) ? c->tblock : 1;
    const std::vector<uint8_t> plan = plan_passes(c->geo, c->til, c->partial_cap, c->step, nsteps, T, want ? K : 0);

    void* pi_cur = c->pi;
    void* pi_oth = c->pi_alt;
    int64_t pending = 0, written = 0;
    // launch timing: a run of consecutive pass-kernel launches (T steps, no
    // diagnostics) is bracketed by one event pair
    size_t spans = 0;
    bool open = false;
    for (uint8_t L : plan) {
        const int64_t n = c->step;
        const bool diag = want && (n % K == 0);
        if (c->lt_on) {
            const bool dom = !diag && L == T;
            if (dom && !open) {
                if (2 * spans + 2 > c->lt_ev.size()) {
                    for (int j = 0; j < 2; ++j) {
                        hipEvent_t e;
                        HIP_TRY(hipEventCreate(&e), "timing event");
                        c->lt_ev.push_back(e);
                    }
                    c->lt_count.push_back(0);
                }
                HIP_TRY(hipEventRecord(c->lt_ev[2 * spans], c->stream), "timing event");
                c->lt_count[spans] = 0;
                open = true;
            } else if (!dom && open) {
                HIP_TRY(hipEventRecord(c->lt_ev[2 * spans + 1], c->stream), "timing event");
                ++spans;
                open = false;
            }
            if (dom) ++c->lt_count[spans];
        }
        WavePartial* parts = diag ? c->partials : nullptr;
        const DiagCoef dc = diag_coef(c, n);
        int64_t ntiles = tc.ntiles;
        if (L > 1) {
            StepCoef64 k[kMaxPassSteps];
            for (int i = 0; i < L; ++i) k[i] = coef_for(c, n + i);
            HIP_TRY(launch_tb(L, c->geo, c->til, c->phi[c->cur], c->phi[c->cur ^ 1], pi_cur, pi_oth, k, diag,
                                parts, dc, c->stream),
                    "multi-step kernel launch");
            std::swap(pi_cur, pi_oth);
            ntiles = tb_tiles(c->geo, c->til, L);
        } else {
            HIP_TRY(launch_step(c->geo, c->til, c->phi[c->cur], c->phi[c->cur ^ 1], pi_cur, pi_cur,
                                coef_for(c, n), true, diag, parts, dc, c->stream),
                    "step kernel launch");
        }
        if (diag) {
            HIP_TRY(launch_finalize(c->partials, ntiles, c->drec + pending, n,
                                    c->p.eta0 + (double)n * c->p.deta, ascale, c->stream),
                    "finalize launch");
            if (++pending == kRecCap) {
                prs_status st = flush(c, pending, series + written);
                if (st != PRS_OK) return st;
                written += pending;
                pending = 0;
            }
        }
        c->cur ^= 1;
        c->step += L;
    }
    if (want) {
        prs_status st = flush(c, pending, series + written);
        if (st != PRS_OK) return st;
        written += pending;
    }
    if (open) {
        HIP_TRY(hipEventRecord(c->lt_ev[2 * spans + 1], c->stream), "timing event");
        ++spans;
    }
    if (spans > 0) {
        HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
        for (size_t i = 0; i < spans; ++i) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, c->lt_ev[2 * i], c->lt_ev[2 * i + 1]), "timing event");
            c->lt_ms += ms;
            c->lt_launches += c->lt_count[i];
        }
    }
    if (n_written) *n_written = written;
    return PRS_OK;
}

prs_status prs_set_launch_timing(prs_ctx* c, int32_t on)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    c->lt_on = on != 0;
    return PRS_OK;
}

prs_status prs_get_launch_timing(prs_ctx* c, double* total_ms, int64_t* launches, int32_t reset)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (total_ms) *total_ms = c->lt_ms;
    if (launches) *launches = c->lt_launches;
    if (reset) {
        c->lt_ms = 0.0;
        c->lt_launches = 0;
    }
    return PRS_OK;
}

prs_status prs_copy(void* dst, const void* src, size_t bytes, void* hip_stream)
{
    if (!dst || !src) return fail(PRS_EINVAL, "NULL buffer");
    if (bytes % 16 != 0 || !aligned16(dst) || !aligned16(src))
        return fail(PRS_EINVAL, "prs_copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    const char* d = static_cast<const char*>(dst);
    const char* r = static_cast<const char*>(src);
    if (d < r + bytes && r < d + bytes) return fail(PRS_EINVAL, "prs_copy buffers overlap");
    HIP_TRY(launch_copy16(src, dst, (int64_t)(bytes / 16), static_cast<hipStream_t>(hip_stream)), "copy launch");
    return PRS_OK;
}

prs_status prs_set_time_blocking(prs_ctx* c, int32_t steps_per_pass)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (steps_per_pass < 1 || steps_per_pass > kMaxPassSteps)
        return fail(PRS_EINVAL, "steps per pass must be 1 .. %d", kMaxPassSteps);
    if (steps_per_pass > 1 && tb_supported(c->geo) && !tb_steps_supported(c->geo, steps_per_pass))
        return fail(PRS_EINVAL, "no %d-step pass kernel for this lattice (2D: 2, 3, 4, 6, 8; "
                    "3D: 2, 3, 4)", steps_per_pass);
    c->tblock = steps_per_pass;
    return PRS_OK;
}

prs_status prs_plan_passes(const prs_ctx* c, int64_t nsteps, int32_t with_records, int64_t* multi_passes,
                           int64_t* single_passes)
{
    if (!c || nsteps < 0) return fail(PRS_EINVAL, "invalid arguments");
    const int T = tb_supported(c->geo) ? c->tblock : 1;
    const int64_t K = (with_records && c->p.diag_every > 0) ? c->p.diag_every : 0;
    int64_t m = 0, n1 = 0;
    for (uint8_t L : plan_passes(c->geo, c->til, c->partial_cap, c->step, nsteps, T, K)) (L > 1 ? m : n1) += 1;
    if (multi_passes) *multi_passes = m;
    if (single_passes) *single_passes = n1;
    return PRS_OK;
}

prs_status prs_get_time_blocking(prs_ctx* c, int32_t* steps_per_pass)
{
    if (!c || !steps_per_pass) return fail(PRS_EINVAL, "NULL argument");
    *steps_per_pass = c->tblock;
    return PRS_OK;
}

prs_status prs_wall_stats(prs_ctx* c, prs_stats* out)
{
    if (!c || !out) return fail(PRS_EINVAL, "NULL argument");
    const TileCounts tc = tile_counts(c->geo, c->til);
    const int64_t n = c->step;
    HIP_TRY(launch_step(c->geo, c->til, c->phi[c->cur], nullptr, c->pi, nullptr, coef_for(c, n), false, true,
                        c->partials, diag_coef(c, n), c->stream),
            "diagnostics kernel launch");
    HIP_TRY(launch_finalize(c->partials, tc.ntiles, c->drec, n, c->p.eta0 + (double)n * c->p.deta,
                            area_scale(c->p), c->stream),
            "finalize launch");
    return flush(c, 1, out);
}

prs_status prs_get_state(prs_ctx* c, void** phi, void** dphi, int64_t* step, double* eta)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (phi) *phi = c->phi[c->cur];
    if (dphi) *dphi = c->pi;
    if (step) *step = c->step;
    if (eta) *eta = c->p.eta0 + (double)c->step * c->p.deta;
    return PRS_OK;
}

prs_status prs_set_state(prs_ctx* c, const void* phi, const void* dphi, int64_t step)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (step < 0) return fail(PRS_EINVAL, "step must be >= 0");
    if ((phi && !aligned16(phi)) || (dphi && !aligned16(dphi)))
        return fail(PRS_EINVAL, "state buffers must be 16-byte aligned");
    const size_t bytes = field_bytes(c->p);
    if (phi && phi != c->phi[c->cur])
        HIP_TRY(hipMemcpyAsync(c->phi[c->cur], phi, bytes, hipMemcpyDeviceToDevice, c->stream), "phi copy");
    if (dphi && dphi != c->pi)
        HIP_TRY(hipMemcpyAsync(c->pi, dphi, bytes, hipMemcpyDeviceToDevice, c->stream), "dphi copy");
    c->step = step;
    return PRS_OK;
}

prs_status prs_set_tiling(prs_ctx* c, int32_t vec, int32_t rows, int32_t ty)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    Tiling t{vec, rows, ty};
    if (!tiling_supported(c->geo, t))
        return fail(PRS_EINVAL, "tiling vec=%d rows=%d ty=%d not supported for this lattice", vec, rows, ty);
    if (tile_counts(c->geo, t).ntiles > c->partial_cap)
        return fail(PRS_EINVAL, "tiling has more wave tiles than the workspace holds (rows >= %lld)",
                    (long long)kMinRows);
    c->til = t;
    return PRS_OK;
}

prs_status prs_set_adjoint_tiling(prs_ctx* c, int32_t vec, int32_t rows, int32_t ty)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    Tiling t{vec, rows, ty};
    if (!tiling_supported(c->geo, t))
        return fail(PRS_EINVAL, "tiling vec=%d rows=%d ty=%d not supported for this lattice", vec, rows, ty);
    if (tile_counts(c->geo, t).ntiles > c->partial_cap)
        return fail(PRS_EINVAL, "tiling has more wave tiles than the workspace holds (rows >= %lld)",
                    (long long)kMinRows);
    c->adj_til = t;
    return PRS_OK;
}

}  // extern "C"

namespace {

// Bytes of the record slot at the start of a slab-diagnostics scratch buffer
// (the wave partials follow it).
constexpr size_t kSlabRecBytes = 256;

// One slab pass; with a record, the diagnostics of its input state: the
// partials go to `scratch`, and the record to the host pointer `record`
// (read back, synchronising the stream) or, with record_on_device, to the
// device pointer `record` (no synchronisation; the record slot of scratch is
// then unused).
prs_status slab_pass(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows, int32_t ty,
                     const void* phi_in, void* phi_out, const void* pi_in, void* pi_out, void* scratch,
                     size_t scratch_bytes, prs_stats* record, void* hip_stream, bool record_on_device = false)
{
    prs_status st = validate(p);
    if (st != PRS_OK) return st;
    if (n0 < 0) return fail(PRS_EINVAL, "n0 must be >= 0");
    if (!phi_in || !phi_out || !pi_in || !pi_out) return fail(PRS_EINVAL, "NULL buffer");
    if (!aligned16(phi_in) || !aligned16(phi_out) || !aligned16(pi_in) || !aligned16(pi_out))
        return fail(PRS_EINVAL, "field buffers must be 16-byte aligned");
    if (phi_in == phi_out || pi_in == pi_out || phi_in == pi_in || phi_out == pi_out)
        return fail(PRS_EINVAL, "the four slab buffers must be distinct");
    const Geometry g = geometry_of(*p);
    const Tiling t{vec, rows, ty};
    if (!tb_supported(g)) return fail(PRS_EUNSUPPORTED, "slab passes need planes shorter than 2^31 bytes");
    if (!tiling_supported(g, t) || !tb_pass_supported(g, t, steps))
        return fail(PRS_EINVAL, "no %d-step %dD pass kernel for vec=%d rows=%d ty=%d", steps, p->ndim, vec, rows,
                    ty);
    const bool diag = record != nullptr;
    const int64_t ntiles = tb_tiles(g, t, steps);
    if (diag) {
        if (!scratch || !aligned16(scratch)) return fail(PRS_EINVAL, "scratch must be a 16-byte aligned buffer");
        const size_t need = kSlabRecBytes + (size_t)ntiles * sizeof(WavePartial);
        if (scratch_bytes < need)
            return fail(PRS_ENOMEM, "slab scratch needs %zu bytes (got %zu)", need, scratch_bytes);
    }
    prs_ctx tmp{};
    tmp.p = *p;
    tmp.V0 = v0_of(*p);
    st = check_stable_until(*p, tmp.V0, n0 + steps - 1);
    if (st != PRS_OK) return st;
    StepCoef64 k[kMaxPassSteps];
    for (int i = 0; i < steps; ++i) k[i] = coef_for(&tmp, n0 + i);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    prs_stats* drec = static_cast<prs_stats*>(scratch);
    WavePartial* parts =
        diag ? reinterpret_cast<WavePartial*>(static_cast<char*>(scratch) + kSlabRecBytes) : nullptr;
    HIP_TRY(launch_tb_slab(steps, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, parts,
                           diag ? diag_coef(&tmp, n0) : DiagCoef{}, s),
            "slab pass launch");
    if (!diag) return PRS_OK;
    HIP_TRY(launch_finalize(parts, ntiles, record_on_device ? record : drec, n0, p->eta0 + (double)n0 * p->deta,
                            area_scale(*p), s),
            "finalize launch");
    if (record_on_device) return PRS_OK;
    HIP_TRY(hipMemcpyAsync(record, drec, sizeof(prs_stats), hipMemcpyDeviceToHost, s), "record copy");
    HIP_TRY(hipStreamSynchronize(s), "record sync");
    return PRS_OK;
}

}  // namespace

extern "C" {

prs_status prs_slab_pass(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows, int32_t ty,
                         const void* phi_in, void* phi_out, const void* pi_in, void* pi_out, void* hip_stream)
{
    return slab_pass(p, n0, steps, vec, rows, ty, phi_in, phi_out, pi_in, pi_out, nullptr, 0, nullptr, hip_stream);
}

size_t prs_slab_scratch_bytes(const prs_params* p, int32_t steps, int32_t vec, int32_t rows, int32_t ty)
{
    if (validate(p) != PRS_OK) return 0;
    const Geometry g = geometry_of(*p);
    const Tiling t{vec, rows, ty};
    if (!tb_supported(g) || !tiling_supported(g, t) || !tb_pass_supported(g, t, steps)) return 0;
    return kSlabRecBytes + (size_t)tb_tiles(g, t, steps) * sizeof(WavePartial);
}

prs_status prs_slab_pass_stats(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows,
                               int32_t ty, const void* phi_in, void* phi_out, const void* pi_in, void* pi_out,
                               void* scratch, size_t scratch_bytes, prs_stats* record, void* hip_stream)
{
    if (!record) return fail(PRS_EINVAL, "record is NULL");
    return slab_pass(p, n0, steps, vec, rows, ty, phi_in, phi_out, pi_in, pi_out, scratch, scratch_bytes, record,
                     hip_stream);
}

prs_status prs_slab_pass_stats_static(const prs_params* p, int64_t n0, int32_t steps, int32_t vec, int32_t rows,
                                      int32_t ty, const void* phi_in, void* phi_out, const void* pi_in,
                                      void* pi_out, prs_stats* record_dev, void* hip_stream)
{
    if (!record_dev || !aligned16(record_dev)) return fail(PRS_EINVAL, "record_dev must be a 16-byte aligned device pointer");
    // the scratch of the stream's device, made current for the look-up
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipDevice_t dev = 0;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "device query");
    HIP_TRY(hipStreamGetDevice(s, &dev), "stream device query");
    if ((int)dev != cur) HIP_TRY(hipSetDevice((int)dev), "set device");
    void* scratch = nullptr;
    size_t bytes = 0;
    hipError_t e = static_scratch(&scratch, &bytes);
    if ((int)dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    const size_t need = prs_slab_scratch_bytes(p, steps, vec, rows, ty);
    if (need == 0) return slab_pass(p, n0, steps, vec, rows, ty, phi_in, phi_out, pi_in, pi_out, nullptr, 0,
                                    record_dev, hip_stream, true);   // reports the invalid argument
    if (need > bytes)
        return fail(PRS_ENOMEM, "the pass has %lld wave tiles; the static scratch holds %lld (%zu bytes, %zu needed)",
                    (long long)((need - kSlabRecBytes) / sizeof(WavePartial)),
                    (long long)((bytes - kSlabRecBytes) / sizeof(WavePartial)), bytes, need);
    return slab_pass(p, n0, steps, vec, rows, ty, phi_in, phi_out, pi_in, pi_out, scratch, bytes, record_dev,
                     hip_stream, true);
}

prs_status prs_set_recompute_tiling(prs_ctx* c, int32_t vec, int32_t rows, int32_t ty, int32_t steps_per_pass)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (steps_per_pass == 0) {
        c->rec_tblock = 0;
        return PRS_OK;
    }
    if (steps_per_pass < 1 || steps_per_pass > kMaxPassSteps)
        return fail(PRS_EINVAL, "steps per pass must be 0 .. %d", kMaxPassSteps);
    Tiling t{vec, rows, ty};
    if (!tiling_supported(c->geo, t))
        return fail(PRS_EINVAL, "tiling vec=%d rows=%d ty=%d not supported for this lattice", vec, rows, ty);
    c->rec_til = t;
    c->rec_tblock = steps_per_pass;
    return PRS_OK;
}

prs_status prs_get_recompute_tiling(prs_ctx* c, int32_t* vec, int32_t* rows, int32_t* ty, int32_t* steps_per_pass)
{
    if (!c || !vec || !rows || !ty || !steps_per_pass) return fail(PRS_EINVAL, "NULL argument");
    const Tiling& t = c->rec_tblock > 0 ? c->rec_til : c->til;
    *vec = t.vec;
    *rows = t.rows;
    *ty = t.ty;
    *steps_per_pass = c->rec_tblock > 0 ? c->rec_tblock : c->tblock;
    return PRS_OK;
}

prs_status prs_set_adjoint_time_blocking(prs_ctx* c, int32_t steps_per_pass)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (steps_per_pass < 1 || steps_per_pass > kMaxPassSteps)
        return fail(PRS_EINVAL, "steps per pass must be 1 .. %d", kMaxPassSteps);
    c->adj_tblock = steps_per_pass;
    return PRS_OK;
}

prs_status prs_set_adjoint_scheme(prs_ctx* c, int32_t scheme)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (scheme != PRS_ADJ_STORED && scheme != PRS_ADJ_FUSED) return fail(PRS_EINVAL, "unknown adjoint scheme %d", scheme);
    c->adj_scheme = scheme;
    return PRS_OK;
}

prs_status prs_get_adjoint_scheme(prs_ctx* c, int32_t* scheme)
{
    if (!c || !scheme) return fail(PRS_EINVAL, "NULL argument");
    *scheme = c->adj_scheme;
    return PRS_OK;
}

prs_status prs_get_adjoint_time_blocking(prs_ctx* c, int32_t* steps_per_pass)
{
    if (!c || !steps_per_pass) return fail(PRS_EINVAL, "NULL argument");
    *steps_per_pass = c->adj_tblock;
    return PRS_OK;
}

prs_status prs_get_adjoint_tiling(prs_ctx* c, int32_t* vec, int32_t* rows, int32_t* ty)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (vec) *vec = c->adj_til.vec;
    if (rows) *rows = c->adj_til.rows;
    if (ty) *ty = c->adj_til.ty;
    return PRS_OK;
}

prs_status prs_get_tiling(prs_ctx* c, int32_t* vec, int32_t* rows, int32_t* ty)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (vec) *vec = c->til.vec;
    if (rows) *rows = c->til.rows;
    if (ty) *ty = c->til.ty;
    return PRS_OK;
}

void prs_destroy(prs_ctx* c)
{
    if (!c) return;
    if (c->hrec) (void)hipHostFree(c->hrec);
    if (c->adj_host) (void)hipHostFree(c->adj_host);
    if (c->adj_aux) {
        (void)hipStreamDestroy(c->adj_aux);
        for (hipEvent_t e : c->adj_ev) (void)hipEventDestroy(e);
    }
    for (hipEvent_t e : c->lt_ev) (void)hipEventDestroy(e);
    delete c;
}

prs_status prs_fill_uniform(void* phi, int64_t count, uint64_t seed, void* hip_stream)
{
    if (count < 0) return fail(PRS_EINVAL, "count must be >= 0");
    if (count > 0 && !phi) return fail(PRS_EINVAL, "phi is NULL");
    HIP_TRY(launch_fill_uniform(phi, count, seed, false, static_cast<hipStream_t>(hip_stream)),
            "fill kernel launch");
    return PRS_OK;
}

prs_status prs_fill_uniform_f64(void* phi, int64_t count, uint64_t seed, void* hip_stream)
{
    if (count < 0) return fail(PRS_EINVAL, "count must be >= 0");
    if (count > 0 && !phi) return fail(PRS_EINVAL, "phi is NULL");
    HIP_TRY(launch_fill_uniform(phi, count, seed, true, static_cast<hipStream_t>(hip_stream)),
            "fill kernel launch");
    return PRS_OK;
}

prs_status prs_fit_scaling(const prs_stats* series, int64_t count, double eta_min, double eta_max,
                           double* mu, double* nu)
{
    if (!series || count < 0 || !mu || !nu) return fail(PRS_EINVAL, "invalid fit arguments");
    // least-squares slope of ln y against ln eta over the selected records
    // (two passes, centred, for accuracy)
    auto slope = [&](bool area) {
        std::vector<double> lx, ly;
        for (int64_t i = 0; i < count; ++i) {
            const prs_stats& r = series[i];
            const double y = area ? r.area_density : r.gv2;
            if (!(r.eta >= eta_min && r.eta <= eta_max && y > 0 && r.eta > 0)) continue;
            lx.push_back(std::log(r.eta));
            ly.push_back(std::log(y));
        }
        const size_t k = lx.size();
        if (k < 2) return std::nan("");
        double mx = 0, my = 0;
        for (size_t i = 0; i < k; ++i) { mx += lx[i]; my += ly[i]; }
        mx /= (double)k;
        my /= (double)k;
        double sxy = 0, sxx = 0;
        for (size_t i = 0; i < k; ++i) {
            sxy += (lx[i] - mx) * (ly[i] - my);
            sxx += (lx[i] - mx) * (lx[i] - mx);
        }
        return sxx > 0 ? sxy / sxx : std::nan("");
    };
    *mu = slope(true);
    *nu = 0.5 * slope(false);   // gamma v = sqrt((gamma v)^2)
    return PRS_OK;
}

}  // extern "C"

namespace {

// Workspace of the checkpointed adjoint (all offsets 256-byte aligned):
//   nseg checkpoints of (phi, phi_dot), the K-1 recomputed fields phi^{n_s+1..}
//   of one segment, two phi_dot scratch fields for the recomputation, mu (x2),
//   w (x2), the per-wave dL/dV0 accumulators, the loss partials and two FP64
//   scalars.
struct AdjLayout {
    size_t fb;
    int64_t nseg, K;
    size_t ck_phi, ck_pi, seg, seg2, pis, pis2, mu, mu2, w0, w1, gacc, lpart, scal, total;
};

constexpr int kSeedBlocks = 1024;

AdjLayout adj_layout(const prs_params& p, int64_t nsteps, int64_t K, int64_t partial_cap)
{
    AdjLayout L;
    L.fb = align_up(field_bytes(p));
    L.K = K;
    L.nseg = (nsteps + K - 1) / K;
    size_t o = 0;
    L.ck_phi = o; o += L.fb * (size_t)L.nseg;
    L.ck_pi = o; o += L.fb * (size_t)L.nseg;
    L.seg = o; o += L.fb * (size_t)(K > 1 ? K - 1 : 0);
    // with two or more segments a second segment buffer lets the next
    // segment's recomputation run while this one is swept
    L.seg2 = o; o += L.nseg > 1 ? L.fb * (size_t)(K > 1 ? K - 1 : 0) : 0;
    L.pis = o; o += L.fb;
    L.pis2 = o; o += L.fb;
    L.mu = o; o += L.fb;
    L.mu2 = o; o += L.fb;
    L.w0 = o; o += L.fb;
    L.w1 = o; o += L.fb;
    L.gacc = o; o += align_up((size_t)partial_cap * sizeof(double));
    L.lpart = o; o += align_up((size_t)kSeedBlocks * sizeof(double));
    L.scal = o; o += align_up(2 * sizeof(double));
    L.total = o;
    return L;
}

template <class T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

prs_status check_adj_args(const prs_ctx* c, int64_t nsteps, int32_t K)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (nsteps < 1) return fail(PRS_EINVAL, "adjoint needs nsteps >= 1");
    if (K < 1) return fail(PRS_EINVAL, "checkpoint interval must be >= 1");
    return PRS_OK;
}

AdjCoef64 adj_coef(const prs_ctx* c, int64_t n, bool last)
{
    const prs_params& p = c->p;
    const double eta = p.eta0 + (double)n * p.deta;
    const double delta = 0.5 * p.alpha * (p.deta / eta) * p.m;
    const double b = p.deta / (1.0 + delta);
    const double kc = 1.0 / (p.phi0 * p.phi0);
    AdjCoef64 k;
    k.a = (1.0 - delta) / (1.0 + delta);
    k.b = b;
    k.cw = last ? 0.0 : p.deta;
    const double A = force_scale(p, n);
    k.F = 4.0 * c->V0 * kc * A;
    k.kc = kc;
    k.inv_dx2 = 1.0 / (p.dx * p.dx);
    k.gscale = -4.0 * kc * b * A;
    return k;
}

}  // namespace

extern "C" {

size_t prs_adjoint_workspace_bytes(const prs_params* p, int64_t nsteps, int32_t ckpt_every)
{
    if (validate(p) != PRS_OK || nsteps < 1 || ckpt_every < 1) return 0;
    return adj_layout(*p, nsteps, ckpt_every, partial_capacity(geometry_of(*p))).total;
}

prs_status prs_adjoint_forward(prs_ctx* c, int64_t nsteps, int32_t ckpt_every, void* work,
                               size_t work_bytes, double* loss)
{
    prs_status st = check_adj_args(c, nsteps, ckpt_every);
    if (st != PRS_OK) return st;
    st = check_stable_until(c->p, c->V0, c->step + nsteps - 1);
    if (st != PRS_OK) return st;
    if (!work || ((uintptr_t)work % kAlign) != 0) return fail(PRS_EINVAL, "work must be 256-byte aligned");
    const AdjLayout L = adj_layout(c->p, nsteps, ckpt_every, c->partial_cap);
    if (work_bytes < L.total)
        return fail(PRS_ENOMEM, "adjoint workspace too small: %zu bytes given, %zu needed", work_bytes, L.total);
    if (!c->adj_host) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->adj_host), 2 * sizeof(double), hipHostMallocDefault),
                "pinned scalars");
    }
    c->adj_ready = false;
    const size_t bytes = field_bytes(c->p);
    const int64_t n0 = c->step;
    // Checkpoint 0 is a copy of the starting state.  Checkpoint s >= 1 is
    // written directly by the pass that ends on it, and the next pass reads
    // it from there, so no further copies are made.  Passes take the run's
    // steps per pass and never cross a checkpoint.
    HIP_TRY(hipMemcpyAsync(at<char>(work, L.ck_phi), c->phi[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream),
            "checkpoint copy");
    HIP_TRY(hipMemcpyAsync(at<char>(work, L.ck_pi), c->pi, bytes, hipMemcpyDeviceToDevice, c->stream),
            "checkpoint copy");
    const int T = tb_supported(c->geo) ? c->tblock : 1;
    const void* phi_in = c->phi[c->cur];
    const void* pi_in = c->pi;
    int64_t k = 0;
    for (uint8_t Lp : plan_passes(c->geo, c->til, c->partial_cap, 0, nsteps, T, L.K)) {
        const int64_t n = n0 + k;
        const bool ck = (k + Lp) % L.K == 0 && k + Lp < nsteps;   // ends on checkpoint (k+Lp)/K
        void* phi_out;
        void* pi_out;
        if (ck) {
            const int64_t sg = (k + Lp) / L.K;
            phi_out = at<char>(work, L.ck_phi + L.fb * sg);
            pi_out = at<char>(work, L.ck_pi + L.fb * sg);
        } else {
            phi_out = c->phi[c->cur ^ 1];
            if (Lp > 1) pi_out = pi_in == c->pi ? c->pi_alt : c->pi;
            else pi_out = (pi_in == c->pi || pi_in == c->pi_alt) ? const_cast<void*>(pi_in) : c->pi;
        }
        if (Lp > 1) {
            StepCoef64 kk[kMaxPassSteps];
            for (int i = 0; i < Lp; ++i) kk[i] = coef_for(c, n + i);
            HIP_TRY(launch_tb(Lp, c->geo, c->til, phi_in, phi_out, pi_in, pi_out, kk, false, nullptr, DiagCoef{},
                              c->stream),
                    "multi-step kernel launch");
        } else {
            HIP_TRY(launch_step(c->geo, c->til, phi_in, phi_out, pi_in, pi_out, coef_for(c, n), true, false,
                                nullptr, DiagCoef{}, c->stream),
                    "step kernel launch");
        }
        if (phi_out == c->phi[c->cur ^ 1]) c->cur ^= 1;
        phi_in = phi_out;
        pi_in = pi_out;
        k += Lp;
        c->step += Lp;
    }
    if (pi_in != c->pi)
        HIP_TRY(hipMemcpyAsync(c->pi, pi_in, bytes, hipMemcpyDeviceToDevice, c->stream), "phi_dot copy");
    const double kc = 1.0 / (c->p.phi0 * c->p.phi0);
    HIP_TRY(launch_adj_seed(c->geo, c->phi[c->cur], sites_of(c->p), kc, c->p.deta, at<char>(work, L.mu),
                            at<char>(work, L.w0), at<double>(work, L.lpart), kSeedBlocks, c->stream),
            "adjoint seed launch");
    HIP_TRY(launch_sum_f64(at<double>(work, L.lpart), kSeedBlocks, at<double>(work, L.scal), c->stream),
            "loss reduce launch");
    HIP_TRY(hipMemcpyAsync(c->adj_host, at<double>(work, L.scal), sizeof(double), hipMemcpyDeviceToHost,
                           c->stream), "loss copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    if (loss) *loss = c->adj_host[0];
    c->adj_ready = true;
    c->adj_n0 = n0;
    c->adj_nsteps = nsteps;
    c->adj_K = ckpt_every;
    c->adj_work = work;
    c->adj_bytes = work_bytes;
    return PRS_OK;
}

namespace {

// Longest pass of at most min(T, left) steps that the adjoint's multi-step
// kernels (the reverse sweep's, else the recomputation's) support with tiling
// t and at most `cap` wave tiles (1: single steps).
int adj_pass_len(const Geometry& g, const Tiling& t, int64_t cap, int T, int64_t left, bool reverse)
{
    int L = (int)std::min<int64_t>(T, left);
    while (L > 1 && !((reverse ? tba_supported(g, t, L) : tb_all_supported(g, t, L)) && tb_tiles(g, t, L) <= cap))
        --L;
    return std::max(L, 1);
}

}  // namespace

}  // extern "C"

namespace {

// The second stream and events of the backward (the recomputation of the
// next-older segment runs on it beside the reverse sweep), created on first
// use on the device of the context's stream, at the default priority.
prs_status adj_aux_ready(prs_ctx* c)
{
    if (c->adj_aux) return PRS_OK;
    int cur = 0;
    hipDevice_t dev = 0;
    HIP_TRY(hipGetDevice(&cur), "device query");
    HIP_TRY(hipStreamGetDevice(c->stream, &dev), "stream device query");
    HIP_TRY(hipSetDevice((int)dev), "set device");
    hipError_t e = hipStreamCreateWithFlags(&c->adj_aux, hipStreamNonBlocking);
    for (hipEvent_t& ev : c->adj_ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        if (c->adj_aux) (void)hipStreamDestroy(c->adj_aux);
        for (hipEvent_t& ev : c->adj_ev) {
            if (ev) (void)hipEventDestroy(ev);
            ev = nullptr;
        }
        c->adj_aux = nullptr;
        return hip_fail(e, "stream/event create");
    }
    return PRS_OK;
}

}  // namespace

extern "C" {

prs_status prs_adjoint_backward(prs_ctx* c, void* work, size_t work_bytes, void* grad_phi0, void* grad_dphi0,
                                double* grad_W0)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (!c->adj_ready || work != c->adj_work || work_bytes != c->adj_bytes)
        return fail(PRS_ESTATE, "prs_adjoint_backward needs the workspace of a preceding prs_adjoint_forward");
    if ((grad_phi0 && !aligned16(grad_phi0)) || (grad_dphi0 && !aligned16(grad_dphi0)))
        return fail(PRS_EINVAL, "gradient buffers must be 16-byte aligned");
    const AdjLayout L = adj_layout(c->p, c->adj_nsteps, c->adj_K, c->partial_cap);
    const int64_t n0 = c->adj_n0;
    const size_t bytes = field_bytes(c->p);
    // the recomputation: its own tuned tiling and pass length, else the forward's
    const Tiling rt = c->rec_tblock > 0 ? c->rec_til : c->til;
    const int T = tb_supported(c->geo) ? (c->rec_tblock > 0 ? c->rec_tblock : c->tblock) : 1;
    const int TA = tb_supported(c->geo) ? c->adj_tblock : 1;
    // The fused scheme (2D): per segment the recomputation keeps only the
    // states at the starts of the reverse passes (TF steps apart, the last
    // pass may be shorter), and each reverse pass recomputes its fields from
    // its pass-start state.  Else every step's field is recomputed and stored.
    const int TF = std::min(TA, 4);
    const bool fused = c->adj_scheme == PRS_ADJ_FUSED && c->geo.ndim == 2 && tb_supported(c->geo) && TF >= 2 &&
                       tbf_supported(c->geo, c->adj_til, TF) &&
                       tbf_tiles(c->geo, c->adj_til, TF) <= c->partial_cap &&
                       tb_pass_supported(c->geo, rt, TF);
    double* gacc = at<double>(work, L.gacc);
    HIP_TRY(launch_zero_f64(gacc, c->partial_cap, c->stream), "zero launch");
    char* mu = at<char>(work, L.mu);
    char* mu_oth = at<char>(work, L.mu2);
    char* wcur = at<char>(work, L.w0);
    char* wnxt = at<char>(work, L.w1);
    char* pis = at<char>(work, L.pis);
    char* pis2 = at<char>(work, L.pis2);
    // phi^{ns+k} of segment sg (k = 1 .. len-1) in its segment buffer
    auto seg_at = [&](int64_t sg, int64_t k) {
        return at<char>(work, ((sg & 1) ? L.seg2 : L.seg) + L.fb * (size_t)(k - 1));
    };
    auto seg_len = [&](int64_t sg) { return std::min<int64_t>(L.K, c->adj_nsteps - sg * L.K); };

    // fused scheme: field f of segment sg's buffer (pass-start state q >= 1
    // holds phi in field 2(q-1) and phi_dot in field 2(q-1)+1)
    auto seg_field = [&](int64_t sg, int64_t f) {
        return at<char>(work, ((sg & 1) ? L.seg2 : L.seg) + L.fb * (size_t)f);
    };
    auto pass_start = [&](int64_t sg, int64_t q, bool pi) -> char* {
        if (q == 0) return at<char>(work, (pi ? L.ck_pi : L.ck_phi) + L.fb * sg);
        return seg_field(sg, 2 * (q - 1) + (pi ? 1 : 0));
    };

    // recompute phi^{ns+1 .. ns+len-1} of segment sg from its checkpoint on
    // stream s: multi-step passes store every step's field; phi_dot goes to
    // the scratch fields.  Fused: TF-step forward passes store the states
    // at the reverse passes' starts instead.
    auto recompute = [&](int64_t sg, hipStream_t s) -> prs_status {
        const int64_t ns = n0 + sg * L.K;
        if (fused) {
            const int64_t len = seg_len(sg);
            const int64_t Q = (len + TF - 1) / TF;
            // forward passes of 2 TF steps that also store their middle
            // state give two pass starts each; a last single one TF steps
            const bool mid = tb_mid_supported(c->geo, rt, 2 * TF);
            for (int64_t q = 0; q + 1 < Q;) {
                StepCoef64 kk[kMaxPassSteps];
                if (mid && q + 2 < Q) {
                    for (int i = 0; i < 2 * TF; ++i) kk[i] = coef_for(c, ns + q * TF + i);
                    HIP_TRY(launch_tb_mid(2 * TF, c->geo, rt, pass_start(sg, q, false), pass_start(sg, q + 2, false),
                                          pass_start(sg, q, true), pass_start(sg, q + 2, true),
                                          pass_start(sg, q + 1, false), pass_start(sg, q + 1, true), kk, s),
                            "recompute launch");
                    q += 2;
                } else {
                    for (int i = 0; i < TF; ++i) kk[i] = coef_for(c, ns + q * TF + i);
                    HIP_TRY(launch_tb(TF, c->geo, rt, pass_start(sg, q, false), pass_start(sg, q + 1, false),
                                      pass_start(sg, q, true), pass_start(sg, q + 1, true), kk, false, nullptr,
                                      DiagCoef{}, s),
                            "recompute launch");
                    q += 1;
                }
            }
            return PRS_OK;
        }
        const int64_t len = seg_len(sg);
        const void* prev = at<char>(work, L.ck_phi + L.fb * sg);
        const void* ckpi = at<char>(work, L.ck_pi + L.fb * sg);
        const void* pprev = ckpi;
        for (int64_t k = 0; k < len - 1;) {
            const int Lp = adj_pass_len(c->geo, rt, c->partial_cap, T, len - 1 - k, false);
            if (Lp > 1) {
                void* outs[kMaxPassSteps];
                StepCoef64 kk[kMaxPassSteps];
                for (int i = 0; i < Lp; ++i) {
                    outs[i] = seg_at(sg, k + 1 + i);
                    kk[i] = coef_for(c, ns + k + i);
                }
                void* pout = pprev == pis ? pis2 : pis;
                HIP_TRY(launch_tb_all(Lp, c->geo, rt, prev, outs, pprev, pout, kk, s), "recompute launch");
                pprev = pout;
            } else {
                void* pout = pprev == ckpi ? pis : const_cast<void*>(pprev);
                HIP_TRY(launch_step(c->geo, rt, prev, seg_at(sg, k + 1), pprev, pout, coef_for(c, ns + k), true,
                                    false, nullptr, DiagCoef{}, s),
                        "recompute launch");
                pprev = pout;
            }
            k += Lp;
            prev = seg_at(sg, k);
        }
        return PRS_OK;
    };

    // reverse sweep over steps ns+len-1 .. ns of segment sg on the context's stream
    auto sweep = [&](int64_t sg) -> prs_status {
        const int64_t ns = n0 + sg * L.K;
        const int64_t len = seg_len(sg);
        if (fused) {
            const int64_t Q = (len + TF - 1) / TF;
            for (int64_t q = Q - 1; q >= 0; --q) {
                const int64_t st = ns + q * TF;                       // the pass's first step
                const int Lq = (int)std::min<int64_t>(TF, len - q * TF);
                if (Lq > 1) {
                    StepCoef64 kk[kMaxPassSteps];
                    AdjCoef64 cc[kMaxPassSteps];
                    for (int i = 0; i + 1 < Lq; ++i) kk[i] = coef_for(c, st + i);
                    for (int k = 1; k <= Lq; ++k) cc[k - 1] = adj_coef(c, st + Lq - k, st + Lq - k == n0);
                    HIP_TRY(launch_tbf(Lq, c->geo, c->adj_til, pass_start(sg, q, false), pass_start(sg, q, true),
                                       wcur, wnxt, mu, mu_oth, gacc, kk, cc, c->stream),
                            "adjoint launch");
                    std::swap(mu, mu_oth);
                } else {
                    HIP_TRY(launch_adjoint(c->geo, c->adj_til, wcur, wnxt, mu, pass_start(sg, q, false), gacc,
                                           adj_coef(c, st, st == n0), c->stream),
                            "adjoint launch");
                }
                std::swap(wcur, wnxt);
            }
            return PRS_OK;
        }
        char* ckphi = at<char>(work, L.ck_phi + L.fb * sg);
        auto phi_at = [&](int64_t j) -> const void* { return j == 0 ? ckphi : seg_at(sg, j); };   // phi^{ns+j}
        for (int64_t k = len - 1; k >= 0;) {
            const int Lp = adj_pass_len(c->geo, c->adj_til, c->partial_cap, TA, k + 1, true);
            if (Lp > 1) {
                const void* phis[kMaxPassSteps];
                AdjCoef64 cc[kMaxPassSteps];
                for (int i = 0; i < Lp; ++i) {
                    phis[i] = phi_at(k - i);
                    cc[i] = adj_coef(c, ns + k - i, ns + k - i == n0);
                }
                HIP_TRY(launch_tba(Lp, c->geo, c->adj_til, wcur, wnxt, mu, mu_oth, phis, gacc, cc, c->stream),
                        "adjoint launch");
                std::swap(mu, mu_oth);
            } else {
                HIP_TRY(launch_adjoint(c->geo, c->adj_til, wcur, wnxt, mu, phi_at(k), gacc,
                                       adj_coef(c, ns + k, ns + k == n0), c->stream),
                        "adjoint launch");
            }
            std::swap(wcur, wnxt);
            k -= Lp;
        }
        return PRS_OK;
    };

    // Segments newest first.  With two segment buffers the recomputation of
    // segment sg-1 runs on a second stream while segment sg is swept: it
    // waits for the sweep of sg+1 (the last reader of its buffer), and the
    // sweep of sg waits for its own recomputation.  The results do not depend
    // on the overlap (each kernel's inputs are complete when it starts).  Only
    // the fused scheme overlaps: its kernels are bound by arithmetic and leave
    // room for each other, while the stored scheme's recomputation and
    // reverse passes are both bound by HBM and gain nothing side by side, so
    // they run in line on the one stream.
    const bool overlap = L.nseg > 1 && fused;
    if (overlap) {
        prs_status st = adj_aux_ready(c);
        if (st != PRS_OK) return st;
    }
    hipStream_t rs = overlap ? c->adj_aux : c->stream;
    if (overlap) {
        HIP_TRY(hipEventRecord(c->adj_ev[0], c->stream), "event record");
        HIP_TRY(hipStreamWaitEvent(rs, c->adj_ev[0], 0), "stream wait");
    }
    prs_status st = recompute(L.nseg - 1, rs);
    if (st != PRS_OK) return st;
    if (overlap) HIP_TRY(hipEventRecord(c->adj_ev[1 + ((L.nseg - 1) & 1)], rs), "event record");
    for (int64_t sg = L.nseg - 1; sg >= 0; --sg) {
        if (overlap && sg >= 1) {
            if (sg + 1 < L.nseg) HIP_TRY(hipStreamWaitEvent(rs, c->adj_ev[3 + ((sg + 1) & 1)], 0), "stream wait");
            st = recompute(sg - 1, rs);
            if (st != PRS_OK) return st;
            HIP_TRY(hipEventRecord(c->adj_ev[1 + ((sg - 1) & 1)], rs), "event record");
        } else if (!overlap && sg + 1 < L.nseg) {
            // in line: segment sg is recomputed after segment sg+1 is swept
            st = recompute(sg, c->stream);
            if (st != PRS_OK) return st;
        }
        if (overlap) HIP_TRY(hipStreamWaitEvent(c->stream, c->adj_ev[1 + (sg & 1)], 0), "stream wait");
        st = sweep(sg);
        if (st != PRS_OK) return st;
        if (overlap) HIP_TRY(hipEventRecord(c->adj_ev[3 + (sg & 1)], c->stream), "event record");
    }
    if (grad_phi0)
        HIP_TRY(hipMemcpyAsync(grad_phi0, mu, bytes, hipMemcpyDeviceToDevice, c->stream), "gradient copy");
    if (grad_dphi0)
        HIP_TRY(hipMemcpyAsync(grad_dphi0, wcur, bytes, hipMemcpyDeviceToDevice, c->stream), "gradient copy");
    HIP_TRY(launch_sum_f64(gacc, c->partial_cap, at<double>(work, L.scal) + 1, c->stream), "G reduce launch");
    HIP_TRY(hipMemcpyAsync(c->adj_host + 1, at<double>(work, L.scal) + 1, sizeof(double),
                           hipMemcpyDeviceToHost, c->stream), "G copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronize");
    const double G = c->adj_host[1];   // dL/dV0
    if (grad_W0) *grad_W0 = std::isinf(c->p.W0) ? 0.0 : G * (-2.0 * c->V0 / c->p.W0);
    c->adj_ready = false;
    return PRS_OK;
}

prs_status prs_adjoint(prs_ctx* c, int64_t nsteps, int32_t ckpt_every, void* work, size_t work_bytes,
                       void* grad_phi0, void* grad_dphi0, double* grad_W0, double* loss)
{
    prs_status st = prs_adjoint_forward(c, nsteps, ckpt_every, work, work_bytes, loss);
    if (st != PRS_OK) return st;
    return prs_adjoint_backward(c, work, work_bytes, grad_phi0, grad_dphi0, grad_W0);
}

}  // extern "C"


// ------------------------------------------------------- batched ensemble --

struct prs_batch {
    int32_t count;
    std::vector<prs_batch_item> items;
    std::vector<Geometry> geo;
    std::vector<Tiling> til;
    std::vector<int32_t> tblock;        // steps per pass (1: single steps)
    std::vector<int64_t> npasses;       // per item, including the final record pass
    std::vector<int64_t> rec_off;       // count + 1 record offsets
    std::vector<int64_t> part_cap;      // partial capacity per realisation
    std::vector<size_t> coef_off, pass_off, alt_off, part_off;
    hipStream_t stream;
    void* ws;
    size_t ws_bytes;
    size_t off_desc, off_coef, off_pass, off_alt, off_part, off_rec, off_ctl;
    size_t off_phase, off_poff, off_ents, off_entp, off_qstart;
    int64_t max_phases;                  // room for this many ticket counters of per-phase launches
    int64_t max_rounds;                  // room for this many rounds in the tables
    int64_t max_ents;                    // room for this many round entries
    int32_t tables_seq;                  // sequences the uploaded tables were built with (-1: none)
    int64_t ctl_count;                   // 32-bit counters of the ensemble kernel
    int64_t total_recs;
    int64_t nphase;                      // rounds of the uploaded tables
    std::vector<int64_t> phase_items;    // items of each round (all queues)
    prs_stats* hrec;     // pinned
    int* herr;           // pinned
    int32_t mode;
    int grid_blocks;
    uint64_t timeout_ticks;
    bool dirty;          // persistent-mode descriptors need uploading
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t capture;  // private stream the graph is captured on (the
                          // caller's stream may be the legacy NULL stream,
                          // which cannot be captured)
    int32_t graph_mode;   // mode the graph was captured for
    std::vector<hipStream_t> workers;   // concurrent streams (STREAMS modes)
    hipEvent_t ev_fork;
    std::vector<hipEvent_t> ev_join;
};

namespace {

struct PassEntry {
    int32_t first, steps, rec, alt;
};

struct BatchLayout {
    size_t desc, coef, pass, alt, part, rec, phase, poff, ents, entp, qstart, ctl, total;
    std::vector<size_t> coef_off, pass_off, alt_off, part_off;
    std::vector<int64_t> rec_off, part_cap;
    int64_t max_phases, max_rounds, max_ents, ctl_count;
};

int64_t batch_records_of(const prs_batch_item& it)
{
    return prs_records_in(&it.p, 0, it.nsteps) + 1;   // + the final state
}

prs_status batch_layout(const prs_batch_item* items, int32_t count, BatchLayout& L)
{
    if (!items || count < 1) return fail(PRS_EINVAL, "batch needs at least one item");
    for (int32_t r = 0; r < count; ++r) {
        prs_status st = validate(&items[r].p);
        if (st != PRS_OK) {
            char why[sizeof g_err];
            std::snprintf(why, sizeof why, "%s", g_err);
            return fail(st, "batch item %d: %s", r, why);
        }
        if (items[r].nsteps < 0) return fail(PRS_EINVAL, "batch item %d: nsteps < 0", r);
        if (items[r].nsteps > 0x3fffffff) return fail(PRS_EINVAL, "batch item %d: too many steps", r);
    }
    // tables of the persistent ensemble kernel: a pass plan has at most
    // nsteps + 1 entries (the last one the final diagnostics)
    size_t o = align_up(sizeof(EnsDesc) * (size_t)count);
    L.desc = 0;
    L.coef = o;
    L.coef_off.assign(count, 0);
    int64_t max_passes = 1, all_passes = 0;
    for (int32_t r = 0; r < count; ++r) {
        L.coef_off[r] = o - L.coef;
        o += align_up((size_t)(items[r].nsteps + 1) * sizeof(EnsCoef));
        max_passes = std::max<int64_t>(max_passes, items[r].nsteps + 1);
        all_passes += items[r].nsteps + 1;
    }
    L.pass = o;
    L.pass_off.assign(count, 0);
    for (int32_t r = 0; r < count; ++r) {
        L.pass_off[r] = o - L.pass;
        o += align_up((size_t)(items[r].nsteps + 1) * sizeof(EnsPass));
    }
    L.max_phases = max_passes;
    L.max_rounds = all_passes;
    L.max_ents = all_passes;
    L.phase = o;
    o += align_up((size_t)kEnsQueues * (size_t)(all_passes + 1) * sizeof(int64_t));
    L.poff = o;
    o += align_up((size_t)(all_passes + 1) * sizeof(int32_t));
    L.ents = o;
    o += align_up((size_t)all_passes * sizeof(int32_t));
    L.entp = o;
    o += align_up((size_t)all_passes * sizeof(int32_t));
    L.qstart = o;
    o += align_up((size_t)kEnsQueues * (size_t)all_passes * sizeof(int64_t));
    L.alt = o;
    L.alt_off.assign(count, 0);
    for (int32_t r = 0; r < count; ++r) {
        L.alt_off[r] = o - L.alt;
        o += align_up(field_bytes(items[r].p));
    }
    L.part = o;
    L.part_off.assign(count, 0);
    L.part_cap.assign(count, 0);
    for (int32_t r = 0; r < count; ++r) {
        L.part_cap[r] = partial_capacity(geometry_of(items[r].p));
        L.part_off[r] = o - L.part;
        o += 2 * align_up((size_t)L.part_cap[r] * sizeof(WavePartial));
    }
    L.rec = o;
    L.rec_off.assign(count + 1, 0);
    for (int32_t r = 0; r < count; ++r) L.rec_off[r + 1] = L.rec_off[r] + batch_records_of(items[r]);
    o += align_up((size_t)L.rec_off[count] * sizeof(prs_stats));
    // counters: the error flag, the queues' ticket counters of each launch
    // (the whole run, or one launch per phase), then per realisation the
    // arrivals and the finished passes
    L.ctl = o;
    L.ctl_count = (1 + kEnsQueues * (max_passes + 1) + 2 * (int64_t)count) * kCtlStride;
    o += align_up((size_t)L.ctl_count * sizeof(uint32_t));
    L.total = o;
    return PRS_OK;
}

// Pass table of one realisation: the single-run pass plan (up to T steps
// per pass, no recorded state inside a pass, an even number of multi-step
// passes so phi_dot ends in the caller's buffer), then the diagnostics-only
// pass of the final state.
std::vector<PassEntry> batch_plan(const prs_batch_item& it, const Geometry& g, const Tiling& t, int64_t cap, int T)
{
    const int64_t S = it.nsteps, K = it.p.diag_every;
    std::vector<PassEntry> out;
    int64_t n = 0, rec = 0;
    int alt = 0;
    for (uint8_t L : plan_passes(g, t, cap, 0, S, T, K)) {
        const bool r = K > 0 && n % K == 0;
        out.push_back(PassEntry{(int32_t)n, (int32_t)L, r ? (int32_t)rec++ : -1, alt});
        if (L > 1) alt ^= 1;
        n += L;
    }
    out.push_back(PassEntry{(int32_t)S, 0, (int32_t)rec, alt});   // final state
    return out;
}

void batch_release_graph(prs_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

bool persistent_mode(int32_t mode)
{
    return mode == PRS_BATCH_PERSISTENT_GRAPH || mode == PRS_BATCH_PERSISTENT || mode == PRS_BATCH_PER_STEP;
}

// Most wave tiles any pass of an item can have (single steps and, for T > 1,
// T-step passes), which its partial buffer must hold.
int64_t item_tiles_max(const Geometry& g, const Tiling& t, int T)
{
    int64_t n = tile_counts(g, t).ntiles;
    if (T > 1) n = std::max<int64_t>(n, tb_tiles(g, t, T));
    return n;
}

// Streams the STREAMS modes run on: one per hardware queue a process gets by
// default.  Created once per ensemble, at the default priority.
constexpr int kBatchStreams = 4;

prs_status batch_streams_ready(prs_batch* b)
{
    if (!b->workers.empty()) return PRS_OK;
    const int ns = std::min<int>(kBatchStreams, b->count);
    HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "event create");
    for (int i = 0; i < ns; ++i) {
        hipStream_t w = nullptr;
        hipEvent_t e = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&w, hipStreamNonBlocking), "stream create");
        b->workers.push_back(w);
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create");
        b->ev_join.push_back(e);
    }
    return PRS_OK;
}

// One realisation's launch sequence on a stream, pass by pass: the pass
// table of batch_plan (up to T steps per pass, records on the pass that
// starts at a recorded state, the final state last), with the single-run
// kernels, each record reduced into its slot of the device record array.
struct ItemCursor {
    int32_t item;
    std::vector<PassEntry> plan;
    size_t next;
    prs_ctx coef;            // parameters for the coefficient schedule
};

prs_status batch_item_begin(prs_batch* b, int32_t r, ItemCursor& cur, hipStream_t s)
{
    const prs_batch_item& it = b->items[r];
    cur.item = r;
    cur.plan = batch_plan(it, b->geo[r], b->til[r], b->part_cap[r], b->tblock[r]);
    cur.next = 0;
    cur.coef = prs_ctx{};
    cur.coef.p = it.p;
    cur.coef.V0 = v0_of(it.p);
    if (it.init_from_seed) {
        const int64_t n = sites_of(it.p);
        const bool f64 = it.p.precision == PRS_F64;
        HIP_TRY(launch_fill_uniform(it.phi_a, n, it.seed, f64, s), "fill launch");
        HIP_TRY(launch_zero_f32(static_cast<float*>(it.dphi), f64 ? 2 * n : n, s), "zero launch");
    }
    return PRS_OK;
}

prs_status batch_item_pass(prs_batch* b, ItemCursor& cur, hipStream_t s)
{
    const int32_t r = cur.item;
    const prs_batch_item& it = b->items[r];
    const Geometry& g = b->geo[r];
    const Tiling& t = b->til[r];
    const size_t idx = cur.next++;
    const PassEntry& e = cur.plan[idx];
    char* base = static_cast<char*>(b->ws);
    void* phi[2] = {it.phi_a, it.phi_b};
    void* dphi = it.dphi;
    void* alt = base + b->off_alt + b->alt_off[r];
    void* pi_now = e.alt ? alt : dphi;
    void* pi_next = e.alt ? dphi : alt;
    const bool diag = e.rec >= 0;
    WavePartial* parts = diag ? reinterpret_cast<WavePartial*>(base + b->off_part + b->part_off[r]) : nullptr;
    const int64_t n = e.first;
    const DiagCoef dc = diag_coef(&cur.coef, n);
    void* phi_in = phi[idx & 1];
    void* phi_out = phi[(idx + 1) & 1];
    int64_t ntiles = tile_counts(g, t).ntiles;
    if (e.steps > 1) {
        StepCoef64 k[kMaxPassSteps];
        for (int i = 0; i < e.steps; ++i) k[i] = coef_for(&cur.coef, n + i);
        HIP_TRY(launch_tb(e.steps, g, t, phi_in, phi_out, pi_now, pi_next, k, diag, parts, dc, s),
                "multi-step kernel launch");
        ntiles = tb_tiles(g, t, e.steps);
    } else if (e.steps == 1) {
        HIP_TRY(launch_step(g, t, phi_in, phi_out, pi_now, pi_now, coef_for(&cur.coef, n), true, diag, parts, dc,
                            s),
                "step kernel launch");
    } else {
        HIP_TRY(launch_step(g, t, phi_in, nullptr, pi_now, nullptr, coef_for(&cur.coef, n), false, true, parts, dc,
                            s),
                "diagnostics kernel launch");
    }
    if (diag) {
        prs_stats* recs = reinterpret_cast<prs_stats*>(base + b->off_rec) + b->rec_off[r];
        HIP_TRY(launch_finalize(parts, ntiles, recs + e.rec, n, it.p.eta0 + (double)n * it.p.deta,
                                area_scale(it.p), s),
                "finalize launch");
    }
    return PRS_OK;
}

// The whole ensemble over the worker streams, forked from and joined back
// into `main`: realisations longest-first onto the least loaded stream, the
// launches interleaved across streams in chunks so every stream starts at
// once, then the records to pinned host memory.
prs_status batch_enqueue_streams(prs_batch* b, hipStream_t main)
{
    prs_status st = batch_streams_ready(b);
    if (st != PRS_OK) return st;
    const int ns = (int)b->workers.size();
    HIP_TRY(hipEventRecord(b->ev_fork, main), "fork event");
    for (hipStream_t w : b->workers) HIP_TRY(hipStreamWaitEvent(w, b->ev_fork, 0), "fork wait");

    std::vector<int32_t> order((size_t)b->count);
    for (int32_t r = 0; r < b->count; ++r) order[(size_t)r] = r;
    auto cost = [&](int32_t r) { return (double)sites_of(b->items[r].p) * (double)(b->items[r].nsteps + 1); };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
    std::vector<std::vector<int32_t>> queue((size_t)ns);
    std::vector<double> load((size_t)ns, 0.0);
    for (int32_t r : order) {
        const size_t w = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        queue[w].push_back(r);
        load[w] += cost(r);
    }

    constexpr int kChunk = 16;   // passes per stream per round
    std::vector<ItemCursor> cur((size_t)ns);
    std::vector<size_t> qpos((size_t)ns, 0);
    std::vector<bool> busy((size_t)ns, false);
    bool any = true;
    while (any) {
        any = false;
        for (int w = 0; w < ns; ++w) {
            for (int c = 0; c < kChunk; ++c) {
                if (!busy[(size_t)w]) {
                    if (qpos[(size_t)w] >= queue[(size_t)w].size()) break;
                    st = batch_item_begin(b, queue[(size_t)w][qpos[(size_t)w]++], cur[(size_t)w],
                                          b->workers[(size_t)w]);
                    if (st != PRS_OK) return st;
                    busy[(size_t)w] = true;
                }
                st = batch_item_pass(b, cur[(size_t)w], b->workers[(size_t)w]);
                if (st != PRS_OK) return st;
                if (cur[(size_t)w].next >= cur[(size_t)w].plan.size()) busy[(size_t)w] = false;
            }
            if (busy[(size_t)w] || qpos[(size_t)w] < queue[(size_t)w].size()) any = true;
        }
    }
    for (int w = 0; w < ns; ++w) {
        HIP_TRY(hipEventRecord(b->ev_join[(size_t)w], b->workers[(size_t)w]), "join event");
        HIP_TRY(hipStreamWaitEvent(main, b->ev_join[(size_t)w], 0), "join wait");
    }
    char* base = static_cast<char*>(b->ws);
    HIP_TRY(hipMemcpyAsync(b->hrec, base + b->off_rec, (size_t)b->total_recs * sizeof(prs_stats),
                           hipMemcpyDeviceToHost, main), "record copy");
    return PRS_OK;
}

// Tables of the persistent ensemble kernel, built on the host and copied
// synchronously: per realisation its coefficients (the single run's FP64
// schedule rounded to float32 as a launch rounds it), its single-run pass
// plan with each pass's tile grid and work items, and its descriptor; then
// the phase tables that number the items (phase p: pass p of every
// realisation that has one, realisation by realisation).
prs_status batch_upload(prs_batch* b, int32_t nseq)
{
    char* base = static_cast<char*>(b->ws);
    std::vector<EnsDesc> desc((size_t)b->count);
    std::vector<std::vector<EnsPass>> passes((size_t)b->count);
    int64_t nphase = 0;
    for (int32_t r = 0; r < b->count; ++r) {
        const prs_batch_item& it = b->items[r];
        const Geometry& g = b->geo[r];
        const Tiling& t = b->til[r];
        prs_ctx tmp{};
        tmp.p = it.p;
        tmp.V0 = v0_of(it.p);
        std::vector<EnsCoef> coef((size_t)it.nsteps + 1);
        for (int64_t n = 0; n <= it.nsteps; ++n) {
            const StepCoef k = f32_of(coef_for(&tmp, n));
            coef[(size_t)n] = EnsCoef{k.a, k.b, k.F, 0.0f, diag_coef(&tmp, n).V0};
        }
        EnsCoef* dcoef = reinterpret_cast<EnsCoef*>(base + b->off_coef + b->coef_off[r]);
        HIP_TRY(hipMemcpy(dcoef, coef.data(), coef.size() * sizeof(EnsCoef), hipMemcpyHostToDevice),
                "coefficient upload");
        const std::vector<PassEntry> plan = batch_plan(it, g, t, b->part_cap[r], b->tblock[r]);
        std::vector<EnsPass>& ps = passes[(size_t)r];
        ps.resize(plan.size());
        int64_t cum = 0;
        for (size_t i = 0; i < plan.size(); ++i) {
            EnsPass& e = ps[i];
            e = EnsPass{};
            e.first = plan[i].first;
            e.steps = plan[i].steps;
            e.rec = plan[i].rec;
            e.alt = plan[i].alt;
            ens_pass_grid(g, t, plan[i].steps, e);
            cum += e.items;
            e.cum_end = cum;
        }
        if (cum >= ((int64_t)1 << 32))
            return fail(PRS_EUNSUPPORTED, "batch item %d: %lld work items exceed the 32-bit counters", r,
                        (long long)cum);
        EnsPass* dpass = reinterpret_cast<EnsPass*>(base + b->off_pass + b->pass_off[r]);
        HIP_TRY(hipMemcpy(dpass, ps.data(), ps.size() * sizeof(EnsPass), hipMemcpyHostToDevice),
                "pass table upload");
        b->npasses[r] = (int64_t)plan.size();
        nphase = std::max<int64_t>(nphase, (int64_t)plan.size());
        const StepCoef k0 = f32_of(coef_for(&tmp, 0));
        EnsDesc& d = desc[(size_t)r];
        d = EnsDesc{};
        d.phi[0] = static_cast<float*>(it.phi_a);
        d.phi[1] = static_cast<float*>(it.phi_b);
        d.pi = static_cast<float*>(it.dphi);
        d.pi_alt = reinterpret_cast<float*>(base + b->off_alt + b->alt_off[r]);
        d.coef = dcoef;
        d.passes = dpass;
        d.part = reinterpret_cast<WavePartial*>(base + b->off_part + b->part_off[r]);
        d.recs = reinterpret_cast<prs_stats*>(base + b->off_rec) + b->rec_off[r];
        d.nx = g.nx;
        d.Q = g.Q;
        d.M = g.M;
        d.ndim = g.ndim;
        d.vec = t.vec;
        d.ty = t.ty;
        d.rows = t.rows;
        d.npasses = (int32_t)plan.size();
        d.unit = (k0.inv_dx2 == 1.0f && k0.kc == 1.0f) ? 1 : 0;
        d.deta = k0.deta;
        d.kc = k0.kc;
        d.inv_dx2 = k0.inv_dx2;
        d.eta0 = it.p.eta0;
        d.deta64 = it.p.deta;
        d.area_scale = area_scale(it.p);
        d.dkc = diag_coef(&tmp, 0).kc;
    }
    // The order of the items: the realisations are dealt, longest first
    // (sites x steps), onto nseq sequences (the least loaded first; nseq = 0:
    // one sequence per realisation), a sequence runs its realisations' passes
    // one after another, and round k holds the k-th pass of every sequence.
    // With one sequence per realisation round k is phase k (pass k of every
    // realisation); with a few sequences only a few realisations are active
    // at a time, as on concurrent streams.  Per queue, where each entry's
    // slice and each round begin: queue q holds items [q n / Q, (q+1) n / Q)
    // of a pass of n items.
    const int32_t S = nseq > 0 ? std::min<int32_t>(nseq, b->count) : b->count;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> seq((size_t)S);
    {
        std::vector<int32_t> order((size_t)b->count);
        for (int32_t r = 0; r < b->count; ++r) order[(size_t)r] = r;
        auto work = [&](int32_t r) { return (double)sites_of(b->items[r].p) * (double)(b->items[r].nsteps + 1); };
        if (nseq > 0)
            std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work(x) > work(y); });
        std::vector<double> load((size_t)S, 0.0);
        for (int32_t k = 0; k < b->count; ++k) {
            const int32_t r = order[(size_t)k];
            size_t sbest = (size_t)(nseq > 0 ? 0 : r);
            if (nseq > 0)
                for (size_t x = 1; x < (size_t)S; ++x)
                    if (load[x] < load[sbest]) sbest = x;
            load[sbest] += work(r);
            for (int32_t pp = 0; pp < (int32_t)passes[(size_t)r].size(); ++pp) seq[sbest].push_back({r, pp});
        }
    }
    nphase = 0;
    for (const auto& q : seq) nphase = std::max<int64_t>(nphase, (int64_t)q.size());
    if (nphase > b->max_rounds) return fail(PRS_EINVAL, "round table larger than its room");
    const int Q = kEnsQueues;
    std::vector<int32_t> off((size_t)nphase + 1, 0);
    std::vector<int32_t> ent_r, ent_p;
    std::vector<std::vector<int64_t>> qs(Q);
    std::vector<int64_t> pstart((size_t)Q * (size_t)(b->max_rounds + 1), 0);
    std::vector<int64_t> qitems(Q, 0);
    b->phase_items.assign((size_t)nphase, 0);
    for (int64_t k = 0; k < nphase; ++k) {
        off[(size_t)k] = (int32_t)ent_r.size();
        for (int q = 0; q < Q; ++q) pstart[(size_t)q * (size_t)(b->max_rounds + 1) + (size_t)k] = qitems[q];
        for (const auto& sq : seq) {
            if (k >= (int64_t)sq.size()) continue;
            const int32_t r = sq[(size_t)k].first, pp = sq[(size_t)k].second;
            const int64_t n = passes[(size_t)r][(size_t)pp].items;
            ent_r.push_back(r);
            ent_p.push_back(pp);
            for (int q = 0; q < Q; ++q) {
                qs[q].push_back(qitems[q]);
                qitems[q] += (int64_t)(q + 1) * n / Q - (int64_t)q * n / Q;
            }
            b->phase_items[(size_t)k] += n;
        }
    }
    off[(size_t)nphase] = (int32_t)ent_r.size();
    for (int q = 0; q < Q; ++q) {
        pstart[(size_t)q * (size_t)(b->max_rounds + 1) + (size_t)nphase] = qitems[q];
        if (qitems[q] >= ((int64_t)1 << 31))
            return fail(PRS_EUNSUPPORTED, "%lld work items exceed the ticket counter", (long long)qitems[q]);
    }
    if ((int64_t)ent_r.size() > b->max_ents) return fail(PRS_EINVAL, "phase table larger than its room");
    HIP_TRY(hipMemcpy(base + b->off_phase, pstart.data(), pstart.size() * sizeof(int64_t), hipMemcpyHostToDevice),
            "phase table upload");
    HIP_TRY(hipMemcpy(base + b->off_poff, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice),
            "phase table upload");
    HIP_TRY(hipMemcpy(base + b->off_ents, ent_r.data(), ent_r.size() * sizeof(int32_t), hipMemcpyHostToDevice),
            "phase table upload");
    HIP_TRY(hipMemcpy(base + b->off_entp, ent_p.data(), ent_p.size() * sizeof(int32_t), hipMemcpyHostToDevice),
            "phase table upload");
    for (int q = 0; q < Q; ++q)
        HIP_TRY(hipMemcpy(base + b->off_qstart + (size_t)q * (size_t)b->max_ents * sizeof(int64_t), qs[q].data(),
                          qs[q].size() * sizeof(int64_t), hipMemcpyHostToDevice),
                "phase table upload");
    HIP_TRY(hipMemcpy(base + b->off_desc, desc.data(), desc.size() * sizeof(EnsDesc), hipMemcpyHostToDevice),
            "descriptor upload");
    b->nphase = nphase;
    b->tables_seq = nseq;
    return PRS_OK;
}

// The whole ensemble as a sequence on the stream: initial fields, the
// counter reset, then the ensemble kernel (one launch over every item, or
// with PRS_BATCH_PER_STEP one launch per phase), then the records and the
// error flag to pinned host memory.
prs_status batch_enqueue(prs_batch* b, bool per_phase, hipStream_t stream)
{
    char* base = static_cast<char*>(b->ws);
    for (int32_t r = 0; r < b->count; ++r) {
        const prs_batch_item& it = b->items[r];
        if (!it.init_from_seed) continue;
        const int64_t n = sites_of(it.p);
        HIP_TRY(launch_fill_uniform(it.phi_a, n, it.seed, false, stream), "fill launch");
        HIP_TRY(launch_zero_f32(static_cast<float*>(it.dphi), n, stream), "zero launch");
    }
    uint32_t* ctl = reinterpret_cast<uint32_t*>(base + b->off_ctl);
    HIP_TRY(launch_ens_reset(ctl, b->ctl_count, stream), "reset launch");
    const int64_t nphase = b->nphase;
    EnsRun run;
    run.desc = reinterpret_cast<const EnsDesc*>(base + b->off_desc);
    run.pstart = reinterpret_cast<const int64_t*>(base + b->off_phase);
    run.phase_off = reinterpret_cast<const int32_t*>(base + b->off_poff);
    run.ent_r = reinterpret_cast<const int32_t*>(base + b->off_ents);
    run.ent_p = reinterpret_cast<const int32_t*>(base + b->off_entp);
    run.qstart = reinterpret_cast<const int64_t*>(base + b->off_qstart);
    run.err = reinterpret_cast<int32_t*>(ctl);
    run.arrive = ctl + (1 + kEnsQueues * (b->max_phases + 1)) * kCtlStride;
    run.ready = run.arrive + (int64_t)b->count * kCtlStride;
    run.pstride = b->max_rounds + 1;
    run.estride = b->max_ents;
    run.timeout = b->timeout_ticks;
    // every queue needs workgroups: at least one per queue
    auto grid = [&](int64_t items) {
        const int64_t g = std::min<int64_t>(b->grid_blocks, items);
        return (int)std::max<int64_t>(kEnsQueues, (g + kEnsQueues - 1) / kEnsQueues * kEnsQueues);
    };
    if (per_phase) {
        for (int64_t p = 0; p < nphase; ++p) {
            run.ticket = ctl + (1 + kEnsQueues * (1 + p)) * kCtlStride;
            run.pb = (int32_t)p;
            run.pe = (int32_t)p + 1;
            HIP_TRY(launch_ens(run, grid(b->phase_items[(size_t)p]), stream), "ensemble phase launch");
        }
    } else {
        int64_t total = 0;
        for (int64_t n : b->phase_items) total += n;
        run.ticket = ctl + kCtlStride;
        run.pb = 0;
        run.pe = (int32_t)nphase;
        HIP_TRY(launch_ens(run, grid(total), stream), "ensemble launch");
    }
    HIP_TRY(hipMemcpyAsync(b->hrec, base + b->off_rec, (size_t)b->total_recs * sizeof(prs_stats),
                           hipMemcpyDeviceToHost, stream), "record copy");
    HIP_TRY(hipMemcpyAsync(b->herr, ctl, sizeof(int), hipMemcpyDeviceToHost, stream), "flag copy");
    return PRS_OK;
}

}  // namespace

extern "C" {

size_t prs_batch_workspace_bytes(const prs_batch_item* items, int32_t count)
{
    BatchLayout L;
    if (batch_layout(items, count, L) != PRS_OK) return 0;
    return L.total;
}

prs_status prs_batch_create(const prs_batch_item* items, int32_t count, void* workspace, size_t ws_bytes,
                            void* hip_stream, prs_batch** out)
{
    if (!out) return fail(PRS_EINVAL, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    prs_status st = batch_layout(items, count, L);
    if (st != PRS_OK) return st;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return fail(PRS_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(PRS_ENOMEM, "batch workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
    for (int32_t r = 0; r < count; ++r) {
        const prs_batch_item& it = items[r];
        if (!it.phi_a || !it.phi_b || !it.dphi || !aligned16(it.phi_a) || !aligned16(it.phi_b) ||
            !aligned16(it.dphi) || it.phi_a == it.phi_b || it.phi_a == it.dphi || it.phi_b == it.dphi)
            return fail(PRS_EINVAL, "batch item %d: three distinct 16-byte aligned fields required", r);
    }
    prs_batch* b = new (std::nothrow) prs_batch();
    if (!b) return fail(PRS_ENOMEM, "host allocation failed");
    b->count = count;
    b->items.assign(items, items + count);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->ws = workspace;
    b->ws_bytes = ws_bytes;
    b->off_desc = L.desc;
    b->off_coef = L.coef;
    b->off_pass = L.pass;
    b->off_alt = L.alt;
    b->off_part = L.part;
    b->off_rec = L.rec;
    b->off_ctl = L.ctl;
    b->off_phase = L.phase;
    b->off_poff = L.poff;
    b->off_ents = L.ents;
    b->off_entp = L.entp;
    b->off_qstart = L.qstart;
    b->max_phases = L.max_phases;
    b->max_rounds = L.max_rounds;
    b->max_ents = L.max_ents;
    b->tables_seq = -1;
    b->ctl_count = L.ctl_count;
    b->coef_off = L.coef_off;
    b->pass_off = L.pass_off;
    b->alt_off = L.alt_off;
    b->part_off = L.part_off;
    b->part_cap = L.part_cap;
    b->rec_off = L.rec_off;
    b->total_recs = L.rec_off[count];
    b->npasses.assign(count, 0);
    for (int32_t r = 0; r < count; ++r) {
        b->geo.push_back(geometry_of(items[r].p));
        Tiling t = default_tiling(b->geo.back());
        t.ty = 1;
        b->til.push_back(t);
        b->tblock.push_back(items[r].p.ndim == 2 && tb_supported(b->geo.back()) ? 2 : 1);
    }
    b->mode = PRS_BATCH_STREAMS;
    b->graph_mode = -1;
    int khz = 0;
    hipError_t e = ens_max_blocks(&b->grid_blocks);
    if (e == hipSuccess) e = batch_clock_rate_khz(&khz);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->hrec),
                                           (size_t)b->total_recs * sizeof(prs_stats), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->herr), sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        prs_batch_destroy(b);
        return hip_fail(e, "batch setup");
    }
    // a pass of the largest realisation takes well under 0.1 s, and a wait
    // never outlasts the pass it waits for; 5 s means something is wrong
    b->timeout_ticks = (uint64_t)(khz > 0 ? khz : 100000) * 1000ull * 5ull;
    b->dirty = true;
    *out = b;
    return PRS_OK;
}

prs_status prs_batch_set_tiling(prs_batch* b, int32_t item, int32_t vec, int32_t rows, int32_t ty)
{
    if (!b || item < 0 || item >= b->count) return fail(PRS_EINVAL, "invalid batch or item");
    Tiling t{vec, rows, ty};
    if (!tiling_supported(b->geo[item], t))
        return fail(PRS_EINVAL, "tiling vec=%d rows=%d ty=%d not available for item %d", vec, rows, ty, item);
    if (item_tiles_max(b->geo[item], t, std::max(2, b->tblock[item])) > b->part_cap[item])
        return fail(PRS_EINVAL, "tiling has more wave tiles than the workspace holds");
    b->til[item] = t;
    batch_release_graph(b);
    b->dirty = true;
    return PRS_OK;
}

prs_status prs_batch_set_time_blocking(prs_batch* b, int32_t item, int32_t steps_per_pass)
{
    if (!b || item < 0 || item >= b->count) return fail(PRS_EINVAL, "invalid batch or item");
    if (steps_per_pass < 1 || steps_per_pass > kMaxPassSteps)
        return fail(PRS_EINVAL, "steps per pass must be 1 .. %d", kMaxPassSteps);
    if (steps_per_pass > 1 && !tb_supported(b->geo[item]))
        return fail(PRS_EUNSUPPORTED, "multi-step passes need rows (2D) shorter than 2^28 sites or planes (3D) "
                    "shorter than 2^31 bytes");
    if (steps_per_pass > 1 && !tb_steps_supported(b->geo[item], steps_per_pass))
        return fail(PRS_EINVAL, "no %d-step pass kernel for this lattice (2D: 2, 3, 4, 6, 8; "
                    "3D: 2, 3, 4)", steps_per_pass);
    if (item_tiles_max(b->geo[item], b->til[item], std::max(2, steps_per_pass)) > b->part_cap[item])
        return fail(PRS_EINVAL, "steps per pass need more wave tiles than the workspace holds");
    b->tblock[item] = steps_per_pass;
    batch_release_graph(b);
    b->dirty = true;
    return PRS_OK;
}

prs_status prs_batch_get_tiling(const prs_batch* b, int32_t item, int32_t* vec, int32_t* rows, int32_t* ty,
                                int32_t* steps_per_pass)
{
    if (!b || item < 0 || item >= b->count) return fail(PRS_EINVAL, "invalid batch or item");
    if (vec) *vec = b->til[item].vec;
    if (rows) *rows = b->til[item].rows;
    if (ty) *ty = b->til[item].ty;
    if (steps_per_pass) *steps_per_pass = b->tblock[item];
    return PRS_OK;
}

prs_status prs_batch_set_mode(prs_batch* b, int32_t mode)
{
    if (!b) return fail(PRS_EINVAL, "batch is NULL");
    if (!persistent_mode(mode) && mode != PRS_BATCH_STREAMS_GRAPH && mode != PRS_BATCH_STREAMS)
        return fail(PRS_EINVAL, "unknown batch mode %d", mode);
    b->mode = mode;
    return PRS_OK;
}

prs_status prs_batch_offsets(const prs_batch* b, int64_t* offsets)
{
    if (!b || !offsets) return fail(PRS_EINVAL, "NULL argument");
    for (int32_t r = 0; r <= b->count; ++r) offsets[r] = b->rec_off[r];
    return PRS_OK;
}

prs_status prs_batch_state(const prs_batch* b, int32_t item, void** phi, void** dphi)
{
    if (!b || item < 0 || item >= b->count) return fail(PRS_EINVAL, "invalid batch or item");
    const prs_batch_item& it = b->items[item];
    const std::vector<PassEntry> plan = batch_plan(it, b->geo[item], b->til[item], b->part_cap[item], b->tblock[item]);
    const int64_t np = (int64_t)plan.size();
    if (phi) *phi = ((np - 1) & 1) ? it.phi_b : it.phi_a;
    if (dphi) *dphi = it.dphi;
    return PRS_OK;
}

prs_status prs_batch_run(prs_batch* b, prs_stats* series, int64_t cap)
{
    if (!b) return fail(PRS_EINVAL, "batch is NULL");
    if (series && cap < b->total_recs)
        return fail(PRS_EINVAL, "series capacity %lld < %lld records", (long long)cap, (long long)b->total_recs);
    const bool persistent = persistent_mode(b->mode);
    for (int32_t r = 0; r < b->count; ++r) {
        const prs_batch_item& it = b->items[r];
        if (it.nsteps > 0) {
            prs_status st = check_stable_until(it.p, v0_of(it.p), it.nsteps - 1);
            if (st != PRS_OK) return st;
        }
    }
    if (persistent) {
        for (int32_t r = 0; r < b->count; ++r)
            if (b->items[r].p.precision != PRS_F32 || !ens_supported(b->geo[r], b->til[r], b->tblock[r]))
                return fail(PRS_EINVAL,
                            "item %d: the persistent modes run float32 items with, in 2D, ty 1 and vec 1 or 2 "
                            "(up to 8 steps per pass) or vec 4 (up to 4); in 3D, single steps with ty 1, or vec 1 "
                            "with ty 8 (up to 4 steps per pass) or ty 16 (up to 3)", r);
    }
    if (b->graph_mode != b->mode) batch_release_graph(b);
    // the per-phase launches keep the phase order (one sequence per
    // realisation); the one-launch modes deal the realisations onto a few
    // sequences
    const int32_t nseq = b->mode == PRS_BATCH_PER_STEP ? 0 : kEnsSequences;
    if (persistent && (b->dirty || b->tables_seq != nseq)) {
        batch_release_graph(b);
        prs_status st = batch_upload(b, nseq);
        if (st != PRS_OK) return st;
        b->dirty = false;
    }
    *b->herr = 0;
    const bool graph = b->mode == PRS_BATCH_PERSISTENT_GRAPH || b->mode == PRS_BATCH_STREAMS_GRAPH;
    if (graph) {
        if (!b->exec) {
            if (!b->capture)
                HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
            if (!persistent) {
                prs_status st = batch_streams_ready(b);
                if (st != PRS_OK) return st;
            }
            HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "graph capture");
            prs_status st = persistent ? batch_enqueue(b, b->mode == PRS_BATCH_PER_STEP, b->capture)
                                       : batch_enqueue_streams(b, b->capture);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->capture, &g);
            if (st != PRS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "graph capture end");
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                batch_release_graph(b);
                return hip_fail(e, "graph instantiate");
            }
            b->graph_mode = b->mode;
        }
        HIP_TRY(hipGraphLaunch(b->exec, b->stream), "graph launch");
    } else if (persistent) {
        prs_status st = batch_enqueue(b, b->mode == PRS_BATCH_PER_STEP, b->stream);
        if (st != PRS_OK) return st;
    } else {
        prs_status st = batch_enqueue_streams(b, b->stream);
        if (st != PRS_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
    if (*b->herr != 0)
        return fail(PRS_EDEVICE, "batched run aborted: a wait of the ensemble kernel timed out");
    if (series) std::memcpy(series, b->hrec, (size_t)b->total_recs * sizeof(prs_stats));
    return PRS_OK;
}

prs_status prs_batch_autotune(prs_batch* b, double* best_ms)
{
    if (!b) return fail(PRS_EINVAL, "batch is NULL");
    for (int32_t r = 0; r < b->count; ++r)
        if (!b->items[r].init_from_seed)
            return fail(PRS_EINVAL, "item %d: the tuner reruns the ensemble, so every item must start from its seed",
                        r);
    // the fastest of two timed runs, after one that uploads the tables and
    // captures the graph of the current settings
    auto time_runs = [&](double* ms) -> prs_status {
        prs_status st = prs_batch_run(b, nullptr, 0);
        double best = 1e300;
        for (int k = 0; k < 2 && st == PRS_OK; ++k) {
            const auto t0 = std::chrono::steady_clock::now();
            st = prs_batch_run(b, nullptr, 0);
            const auto t1 = std::chrono::steady_clock::now();
            best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        *ms = best;
        return st;
    };
    // realisations with the same lattice and the same setting move together
    struct Group {
        std::vector<int32_t> items;
        double work;
    };
    std::vector<Group> groups;
    for (int32_t r = 0; r < b->count; ++r) {
        const Geometry& g = b->geo[r];
        const Tiling& t = b->til[r];
        double work = (double)g.nx * (double)g.Q * (double)g.M * (double)b->items[r].nsteps;
        bool placed = false;
        for (Group& G : groups) {
            const int32_t q = G.items[0];
            const Geometry& h = b->geo[q];
            const Tiling& u = b->til[q];
            if (h.ndim == g.ndim && h.f64 == g.f64 && h.nx == g.nx && h.Q == g.Q && h.M == g.M && u.vec == t.vec &&
                u.rows == t.rows && u.ty == t.ty && b->tblock[q] == b->tblock[r]) {
                G.items.push_back(r);
                G.work += work;
                placed = true;
                break;
            }
        }
        if (!placed) groups.push_back(Group{{r}, work});
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& c) { return a.work > c.work; });
    const bool persistent = persistent_mode(b->mode);
    double best = 0.0;
    prs_status st = time_runs(&best);
    if (st != PRS_OK) return st;
    for (const Group& G : groups) {
        const int32_t q = G.items[0];
        const Geometry& g = b->geo[q];
        // a setting the mode runs and the item's partial buffer holds
        auto usable = [&](const Tiling& t, int T) {
            if (!tiling_supported(g, t) || (T > 1 && !tb_pass_supported(g, t, T))) return false;
            if (persistent && !ens_supported(g, t, T)) return false;
            return item_tiles_max(g, t, std::max(2, T)) <= b->part_cap[q];
        };
        auto apply = [&](const Tiling& t, int T) {
            for (int32_t r : G.items) {
                b->til[r] = t;
                b->tblock[r] = T;
            }
            batch_release_graph(b);
            b->dirty = true;
        };
        for (;;) {
            const Tiling cur = b->til[q];
            const int T = b->tblock[q];
            // candidates: the marching tile doubled (up to the tuner's
            // longest, 128, and not past the lattice); in 3D, when the
            // current tiling is a workgroup-stacked one, the other
            // workgroup shapes, each with the longest pass the mode runs
            std::vector<std::pair<Tiling, int>> cand;
            const Tiling taller{cur.vec, cur.rows * 2, cur.ty};
            if (taller.rows <= 128 && cur.rows < g.M && usable(taller, T)) cand.push_back({taller, T});
            if (g.ndim == 3 && cur.ty >= 8 && T > 1) {
                for (int ty : {8, 16, 32, 64}) {
                    if (ty == cur.ty) continue;
                    const Tiling t{cur.vec, cur.rows, ty};
                    for (int U = 4; U >= 2; --U)
                        if (usable(t, U)) {
                            cand.push_back({t, U});
                            break;
                        }
                }
            }
            double round_best = 1e300;
            size_t pick = cand.size();
            for (size_t c = 0; c < cand.size(); ++c) {
                apply(cand[c].first, cand[c].second);
                double ms = 0.0;
                st = time_runs(&ms);
                if (st != PRS_OK) {
                    apply(cur, T);
                    return st;
                }
                if (ms < round_best) {
                    round_best = ms;
                    pick = c;
                }
            }
            // a change must gain more than the runs' spread to be kept
            if (pick < cand.size() && round_best < best * 0.98) {
                apply(cand[pick].first, cand[pick].second);
                best = round_best;
                continue;
            }
            apply(cur, T);
            break;
        }
    }
    if (best_ms) *best_ms = best;
    return PRS_OK;
}

void prs_batch_destroy(prs_batch* b)
{
    if (!b) return;
    batch_release_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (hipStream_t w : b->workers) (void)hipStreamDestroy(w);
    for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->hrec) (void)hipHostFree(b->hrec);
    if (b->herr) (void)hipHostFree(b->herr);
    delete b;
}

}  // extern "C"

// -------------------------------------------------------------- autotuner --
//
// Candidate tilings are timed on the context's own state (saved and restored
// around every candidate, so the run is unchanged), and the fastest is kept
// and written to a small JSON cache keyed by GPU architecture, dimension,
// lattice size and tiling set.  The paper notes that a new card needs the
// code re-optimised (Sec. IV); this does it per lattice shape.

namespace {

constexpr const char* kTuneVersion = "k4";

std::string tune_key(const prs_params& p, bool batch_set)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|%dD|%lldx%lldx%lld|%s%s|%s", arch.c_str(), p.ndim,
                  (long long)p.n[0], (long long)p.n[1], (long long)(p.ndim == 3 ? p.n[2] : 1),
                  batch_set ? "batch" : "single", p.precision == PRS_F64 ? "|f64" : "", kTuneVersion);
    return buf;
}

struct TuneEntry {
    int vec, rows, ty, tb;
    double us;
};

// The cache is written by tune_write only: one entry per line,
//   "key": {"vec": V, "rows": R, "ty": T, "steps_per_pass": P, "us": U},
std::map<std::string, TuneEntry> tune_read(const char* path)
{
    std::map<std::string, TuneEntry> m;
    FILE* f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return m;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char* q1 = std::strchr(line, '"');
        if (!q1) continue;
        const char* q2 = std::strchr(q1 + 1, '"');
        if (!q2) continue;
        TuneEntry e;
        if (std::sscanf(q2 + 1, ": {\"vec\": %d, \"rows\": %d, \"ty\": %d, \"steps_per_pass\": %d, \"us\": %lf",
                        &e.vec, &e.rows, &e.ty, &e.tb, &e.us) == 5)
            m[std::string(q1 + 1, q2)] = e;
    }
    std::fclose(f);
    return m;
}

bool tune_write(const char* path, const std::map<std::string, TuneEntry>& m)
{
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        std::fprintf(f, "\"%s\": {\"vec\": %d, \"rows\": %d, \"ty\": %d, \"steps_per_pass\": %d, \"us\": %.3f}%s\n",
                     kv.first.c_str(), kv.second.vec, kv.second.rows, kv.second.ty, kv.second.tb, kv.second.us,
                     ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    return std::rename(tmp.c_str(), path) == 0;
}

int device_compute_units()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return ncu;
}

// Row heights that make a pass's workgroup count a whole number of rounds
// over the compute units: for each vec and k = 1 .. kmax, the shortest tile
// (kMinRows .. 128 rows) with at most k workgroups per unit, when the
// setting is usable and not already among `have`.  On lattices whose pass
// has only a few waves per SIMD, a partial last round leaves the units that
// got one workgroup fewer idle while it runs.
template <typename Usable, typename Workgroups>
void add_balanced_rows(std::vector<Tiling>& have, int kmax, int ncu, Usable usable, Workgroups workgroups)
{
    if (ncu <= 0) return;
    for (int vec : {1, 2, 4})
        for (int k = 1; k <= kmax; ++k)
            for (int r = (int)kMinRows; r <= 128; ++r) {
                const Tiling t{vec, r, 1};
                if (!usable(t)) break;
                if (workgroups(t) <= (int64_t)k * ncu) {
                    bool seen = false;
                    for (const Tiling& u : have) seen = seen || (u.vec == t.vec && u.rows == t.rows && u.ty == t.ty);
                    if (!seen) have.push_back(t);
                    break;
                }
            }
}

std::vector<Tiling> tune_candidates(const Geometry& g, bool batch_set)
{
    std::vector<Tiling> out;
    for (int vec : {1, 2, 4})
        for (int rows : {8, 16, 32, 64, 128})
            for (int ty : {1, 2, 4, 8, 16, 32, 64}) {
                Tiling t{vec, rows, ty};
                if (rows < kMinRows && rows < g.M) continue;
                if (!tiling_supported(g, t)) continue;
                if (batch_set && !ens_supported(g, t, 1)) continue;
                out.push_back(t);
            }
    return out;
}

}  // namespace

extern "C" {

prs_status prs_tuned_tiling(const prs_params* p, const char* cache_path, int32_t flags, int32_t* vec,
                            int32_t* rows, int32_t* ty)
{
    prs_status st = validate(p);
    if (st != PRS_OK) return st;
    const auto m = tune_read(cache_path);
    const auto it = m.find(tune_key(*p, (flags & PRS_TUNE_BATCH) != 0));
    if (it == m.end()) return fail(PRS_ESTATE, "no cached tiling for this lattice");
    if (vec) *vec = it->second.vec;
    if (rows) *rows = it->second.rows;
    if (ty) *ty = it->second.ty;
    return PRS_OK;
}

}  // extern "C"

namespace {

// Tunes the reverse-sweep kernel's tiling and steps per pass on scratch
// buffers (w, mu filled from the current phi; phi^n = the current phi).  The
// recomputation keeps following the forward's setting: timing its passes on
// scratch fields that stay cache-resident misjudges them (single steps win
// there and lose by 15 % inside the backward), and the forward's setting
// was within 2 % of the best one measured inside the backward at 2048^2 and
// 256^3.
size_t tune_field_bytes(const prs_ctx* c) { return align_up(field_bytes(c->p)); }

// Least workspace of the adjoint tuner: w and mu twice, one dL/dV0
// accumulator per wave tile.
size_t tune_adjoint_min_bytes(const prs_ctx* c)
{
    return 4 * tune_field_bytes(c) + align_up((size_t)c->partial_cap * sizeof(double));
}

prs_status autotune_adjoint(prs_ctx* c, const char* cache_path, int32_t flags, void* work, size_t work_bytes,
                            double* best_us)
{
    const std::string key = tune_key(c->p, false) + (c->adj_scheme == PRS_ADJ_FUSED ? "|adjoint-fused" : "|adjoint");
    auto cache = tune_read(cache_path);
    if (!(flags & PRS_TUNE_FORCE)) {
        const auto it = cache.find(key);
        if (it != cache.end() &&
            prs_set_adjoint_tiling(c, it->second.vec, it->second.rows, it->second.ty) == PRS_OK &&
            prs_set_adjoint_time_blocking(c, it->second.tb) == PRS_OK) {
            if (best_us) *best_us = it->second.us;
            return PRS_OK;
        }
    }
    const std::vector<Tiling> cand = tune_candidates(c->geo, false);
    const size_t need = tune_adjoint_min_bytes(c);
    if (!work || work_bytes < need)
        return fail(PRS_ENOMEM, "adjoint tuner workspace: %zu bytes given, at least %zu needed", work_bytes, need);
    if (((uintptr_t)work % kAlign) != 0) return fail(PRS_EINVAL, "tuner workspace must be 256-byte aligned");
    const size_t bytes = field_bytes(c->p);
    const size_t fb = tune_field_bytes(c);
    char* buf = static_cast<char*>(work);
    double* gacc = reinterpret_cast<double*>(buf + 4 * fb);
    // Each reverse step reads its own phi^n in the backward; the workspace
    // beyond the least holds up to 32 distinct phi fields that the timed
    // steps read in rotation, more than the last-level cache holds at the
    // lattices the adjoint is run on (one shared field would be served from
    // cache and flatter the multi-step passes, which read T of them per pass).
    char* phis0 = buf + need;
    const int nphi = (int)std::min<size_t>(32, (work_bytes - need) / fb);
    hipError_t e = hipSuccess;
    char* w0 = buf;
    char* w1 = buf + fb;
    char* mu0 = buf + 2 * fb;
    char* mu1 = buf + 3 * fb;
    auto phi_of = [&](int n) -> const void* {
        return nphi > 0 ? static_cast<const void*>(phis0 + (size_t)(n % nphi) * fb) : c->phi[c->cur];
    };
    // With twelve or more fields the fused scheme's reverse passes and its
    // recomputation each rotate through half of them (their own fields, so
    // that the two streams share no data); otherwise both use them all.
    bool split = false;
    auto phi_rev = [&](int n) -> const void* {
        return split ? static_cast<const void*>(phis0 + (size_t)(n % (nphi / 2)) * fb) : phi_of(n);
    };
    auto phi_fwd = [&](int n) -> void* {
        const int h = nphi / 2;
        return const_cast<void*>(split ? static_cast<const void*>(phis0 + (size_t)(h + n % (nphi - h)) * fb)
                                       : phi_of(n));
    };
    if (e == hipSuccess) e = hipMemcpyAsync(w0, c->phi[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(mu0, c->phi[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream);
    for (int i = 0; i < nphi && e == hipSuccess; ++i)
        e = hipMemcpyAsync(phis0 + (size_t)i * fb, c->phi[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = launch_zero_f64(gacc, c->partial_cap, c->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double sites = (double)sites_of(c->p);
    const int timed = (int)std::max(8.0, std::min(48.0, 4e9 / std::max(sites, 1.0)));
    const char* env = std::getenv("PRS_TUNE_LOG");
    const bool log_each = env && env[0] == '1';
    Tiling best = c->adj_til;
    int best_T = 1;
    double best_t = 1e300;
    // Fused scheme (2D): every reverse-pass tiling and length that has a
    // kernel, each timed together with the forward pass that recomputes its
    // pass-start state (the recomputation's tiling) -- what one reverse pass
    // costs inside the backward.
    const Tiling rt = c->rec_tblock > 0 ? c->rec_til : c->til;
    const bool fused = c->adj_scheme == PRS_ADJ_FUSED && c->geo.ndim == 2 && tb_supported(c->geo) && nphi >= 6;
    // Besides the power-of-two row tiles, the heights that give the reverse
    // pass a whole number of workgroup rounds (at 2048^2 it has two or three
    // waves per SIMD).
    const int ncu = device_compute_units();
    if (fused && nphi >= 12) {
        prs_status st = adj_aux_ready(c);
        if (st != PRS_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st;
        }
        split = true;
    }
    for (int T : {2, 3, 4}) {
        if (!fused) break;
        if (!tb_pass_supported(c->geo, rt, T)) continue;
        std::vector<Tiling> fcand = cand;
        add_balanced_rows(
            fcand, 8, ncu, [&](const Tiling& t) { return tbf_supported(c->geo, t, T); },
            [&](const Tiling& t) { return tbf_workgroups(c->geo, t, T); });
        for (const Tiling& t : fcand) {
            if (e != hipSuccess) break;
            if (!tbf_supported(c->geo, t, T) || tbf_tiles(c->geo, t, T) > c->partial_cap) continue;
            char* a = w0;
            char* b = w1;
            char* ma = mu0;
            char* mb = mu1;
            auto run = [&](int steps) -> hipError_t {
                const bool mid = tb_mid_supported(c->geo, rt, 2 * T);
                // as in the backward, the recomputation runs on the second
                // stream beside the reverse passes, on fields of its own
                // (the second half of the rotation), when there are enough
                hipError_t err = hipSuccess;
                if (split) {
                    err = hipEventRecord(c->adj_ev[0], c->stream);
                    if (err == hipSuccess) err = hipStreamWaitEvent(c->adj_aux, c->adj_ev[0], 0);
                }
                for (int k = 0; k < steps && err == hipSuccess; k += T) {
                    StepCoef64 kk[kMaxPassSteps];
                    AdjCoef64 cc[kMaxPassSteps];
                    for (int i = 0; i < 2 * T && i < kMaxPassSteps; ++i) kk[i] = coef_for(c, c->step);
                    for (int i = 0; i < T; ++i) cc[i] = adj_coef(c, c->step, false);
                    // pass-start states and the forward's outputs in rotation;
                    // one forward pass of 2T steps per two reverse passes
                    // where it has a kernel, as in the backward
                    const void* ps = phi_rev(k);
                    const void* pp = phi_rev(k + 1);
                    auto fwd = [&](int i) { return phi_fwd(k + i); };
                    hipStream_t fs = split ? c->adj_aux : c->stream;
                    if (!mid)
                        err = launch_tb(T, c->geo, rt, fwd(0), fwd(2), fwd(1), fwd(3), kk, false, nullptr, DiagCoef{},
                                        fs);
                    else if ((k / T) % 2 == 0)
                        err = launch_tb_mid(2 * T, c->geo, rt, fwd(0), fwd(2), fwd(1), fwd(3), fwd(4), fwd(5), kk, fs);
                    if (err == hipSuccess)
                        err = launch_tbf(T, c->geo, t, ps, pp, a, b, ma, mb, gacc, kk, cc, c->stream);
                    std::swap(a, b);
                    std::swap(ma, mb);
                }
                if (split && err == hipSuccess) {
                    err = hipEventRecord(c->adj_ev[1], c->adj_aux);
                    if (err == hipSuccess) err = hipStreamWaitEvent(c->stream, c->adj_ev[1], 0);
                }
                return err;
            };
            e = run(2 * T);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = run(timed);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const int done = (timed + T - 1) / T * T;
            const double per_step = ms / done;
            if (e == hipSuccess && log_each)
                std::fprintf(stderr, "prs_autotune(adjoint, fused): vec=%d rows=%d steps/pass=%d %.2f us/step\n",
                             t.vec, t.rows, T, per_step * 1e3);
            if (e == hipSuccess && per_step < best_t) {
                best_t = per_step;
                best = t;
                best_T = T;
            }
        }
    }
    // single reverse steps for every tiling; multi-step reverse passes for
    // the tilings and lengths that have kernels (stored scheme)
    for (int T : {1, 2, 3, 4, 8}) {
        if (fused) break;
        for (const Tiling& t : cand) {
            if (e != hipSuccess) break;
            if (tile_counts(c->geo, t).ntiles > c->partial_cap) continue;
            if (T > 1 && !(tb_supported(c->geo) && tba_supported(c->geo, t, T) &&
                           tb_tiles(c->geo, t, T) <= c->partial_cap))
                continue;
            char* a = w0;
            char* b = w1;
            char* ma = mu0;
            char* mb = mu1;
            auto run = [&](int steps) -> hipError_t {
                for (int k = 0; k < steps; k += T) {
                    hipError_t err;
                    if (T > 1) {
                        const void* phis[kMaxPassSteps];
                        AdjCoef64 cc[kMaxPassSteps];
                        for (int i = 0; i < T; ++i) {
                            phis[i] = phi_of(k + i);
                            cc[i] = adj_coef(c, c->step, false);
                        }
                        err = launch_tba(T, c->geo, t, a, b, ma, mb, phis, gacc, cc, c->stream);
                        std::swap(ma, mb);
                    } else {
                        err = launch_adjoint(c->geo, t, a, b, ma, phi_of(k), gacc, adj_coef(c, c->step, false),
                                             c->stream);
                    }
                    if (err != hipSuccess) return err;
                    std::swap(a, b);
                }
                return hipSuccess;
            };
            e = run(2 * T);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = run(timed);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const int done = (timed + T - 1) / T * T;
            const double per_step = ms / done;
            if (e == hipSuccess && log_each)
                std::fprintf(stderr, "prs_autotune(adjoint): vec=%d rows=%d ty=%d steps/pass=%d %.2f us/step\n",
                             t.vec, t.rows, t.ty, T, per_step * 1e3);
            if (e == hipSuccess && per_step < best_t) {
                best_t = per_step;
                best = t;
                best_T = T;
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "adjoint autotune");
    c->adj_til = best;
    c->adj_tblock = best_T;
    if (best_us) *best_us = best_t * 1e3;
    if (cache_path && cache_path[0]) {
        cache[key] = TuneEntry{best.vec, best.rows, best.ty, best_T, best_t * 1e3};
        if (!tune_write(cache_path, cache)) return fail(PRS_EINVAL, "cannot write tuning cache %s", cache_path);
    }
    return PRS_OK;
}

}  // namespace

extern "C" {

size_t prs_tune_workspace_bytes(const prs_ctx* c, int32_t flags)
{
    if (!c) return 0;
    if (flags & PRS_TUNE_ADJOINT)
        return tune_adjoint_min_bytes(c) + ((flags & PRS_TUNE_MIN_WORKSPACE) ? 0 : 32 * tune_field_bytes(c));
    return 2 * tune_field_bytes(c);
}

prs_status prs_autotune(prs_ctx* c, const char* cache_path, int32_t flags, void* work, size_t work_bytes,
                        double* best_us)
{
    if (!c) return fail(PRS_EINVAL, "ctx is NULL");
    if (flags & PRS_TUNE_ADJOINT) return autotune_adjoint(c, cache_path, flags, work, work_bytes, best_us);
    const bool batch_set = (flags & PRS_TUNE_BATCH) != 0;
    const std::string key = tune_key(c->p, batch_set);
    auto cache = tune_read(cache_path);
    if (!(flags & PRS_TUNE_FORCE)) {
        const auto it = cache.find(key);
        if (it != cache.end()) {
            prs_status st = prs_set_tiling(c, it->second.vec, it->second.rows, it->second.ty);
            // the cached steps per pass, also when it is 1 (single steps)
            if (st == PRS_OK) st = prs_set_time_blocking(c, std::max(1, it->second.tb));
            if (st == PRS_OK) {
                if (best_us) *best_us = it->second.us;
                return PRS_OK;
            }
        }
    }
    const std::vector<Tiling> cand = tune_candidates(c->geo, batch_set);
    if (cand.empty()) return fail(PRS_EUNSUPPORTED, "no tiling candidates");
    const size_t bytes = field_bytes(c->p);
    const size_t need = prs_tune_workspace_bytes(c, flags);
    if (!work || work_bytes < need)
        return fail(PRS_ENOMEM, "tuner workspace: %zu bytes given, %zu needed", work_bytes, need);
    if (((uintptr_t)work % kAlign) != 0) return fail(PRS_EINVAL, "tuner workspace must be 256-byte aligned");
    void* save_phi = work;
    void* save_pi = static_cast<char*>(work) + tune_field_bytes(c);
    hipError_t e = hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double sites = (double)sites_of(c->p);
    const int timed = (int)std::max(4.0, std::min(40.0, 4e9 / std::max(sites, 1.0)));
    const int64_t n0 = c->step;
    const int cur0 = c->cur;
    const char* env = std::getenv("PRS_TUNE_LOG");
    const bool log_each = env && env[0] == '1';
    Tiling best = c->til;
    double best_t = 1e300;
    prs_status result = PRS_OK;
    // 2D single runs also choose the steps per pass: a candidate with T > 1
    // is timed on T-step passes and its per-step time is a pass over T
    int per = 1;
    auto run = [&](const Tiling& t, int passes) -> hipError_t {
        void* pa = c->pi;
        void* pb = c->pi_alt;
        for (int k = 0; k < passes; ++k) {
            hipError_t err;
            if (per > 1) {
                StepCoef64 kc[kMaxPassSteps];
                for (int i = 0; i < per; ++i) kc[i] = coef_for(c, n0 + per * k + i);
                err = launch_tb(per, c->geo, t, c->phi[c->cur], c->phi[c->cur ^ 1], pa, pb, kc, false, nullptr,
                                  DiagCoef{}, c->stream);
                std::swap(pa, pb);
            } else {
                err = launch_step(c->geo, t, c->phi[c->cur], c->phi[c->cur ^ 1], c->pi, c->pi,
                                  coef_for(c, n0 + k), true, false, nullptr, DiagCoef{}, c->stream);
            }
            if (err != hipSuccess) return err;
            c->cur ^= 1;
        }
        return hipSuccess;
    };
    const int max_T = tb_supported(c->geo) ? kMaxPassSteps : 1;
    int best_T = c->tblock;
    e = hipMemcpyAsync(save_phi, c->phi[cur0], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(save_pi, c->pi, bytes, hipMemcpyDeviceToDevice, c->stream);
    const int ncu = device_compute_units();
    for (int T = 1; T <= max_T; ++T) {
        if (T > 1 && !tb_steps_supported(c->geo, T)) continue;
        per = T;
        // 2D multi-step passes also try the heights that give a whole number
        // of workgroup rounds, up to four per compute unit (lattices whose
        // pass fills the units many times over get none)
        std::vector<Tiling> tcand = cand;
        if (c->geo.ndim == 2 && T > 1)
            add_balanced_rows(
                tcand, 4, ncu,
                [&](const Tiling& t) {
                    return tb_pass_supported(c->geo, t, T) && (!batch_set || ens_supported(c->geo, t, T));
                },
                [&](const Tiling& t) { return tb2_workgroups(c->geo, t, T); });
        for (const Tiling& t : tcand) {
            if (e != hipSuccess) break;
            if (T > 1 && !tb_pass_supported(c->geo, t, T)) continue;
            if (batch_set && !ens_supported(c->geo, t, T)) continue;
            if (tile_counts(c->geo, t).ntiles > c->partial_cap) continue;
            if (T > 1 && tb_tiles(c->geo, t, T) > c->partial_cap) continue;
            e = run(t, 2);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = run(t, timed);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double per_step = ms / ((double)timed * per);
            if (e == hipSuccess && log_each)
                std::fprintf(stderr, "prs_autotune: vec=%d rows=%d ty=%d steps/pass=%d %.2f us/step\n", t.vec,
                             t.rows, t.ty, per, per_step * 1e3);
            if (e == hipSuccess && per_step < best_t) {
                best_t = per_step;
                best = t;
                best_T = T;
            }
            // restore the state for the next candidate (and for the caller)
            c->cur = cur0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->phi[cur0], save_phi, bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(c->pi, save_pi, bytes, hipMemcpyDeviceToDevice, c->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) result = hip_fail(e, "autotune");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->cur = cur0;
    c->step = n0;
    if (result != PRS_OK) return result;
    c->til = best;
    c->tblock = best_T;
    if (best_us) *best_us = best_t * 1e3;
    if (cache_path && cache_path[0]) {
        cache[key] = TuneEntry{best.vec, best.rows, best.ty, best_T, best_t * 1e3};
        if (!tune_write(cache_path, cache)) return fail(PRS_EINVAL, "cannot write tuning cache %s", cache_path);
    }
    return PRS_OK;
}

}  // extern "C"

extern "C" {

const char* prs_strerror(prs_status s)
{
    switch (s) {
    case PRS_OK: return "ok";
    case PRS_EINVAL: return "invalid argument";
    case PRS_ENOMEM: return "out of memory or workspace too small";
    case PRS_EDEVICE: return "HIP device error";
    case PRS_ESTATE: return "invalid state for this call";
    case PRS_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* prs_last_error(void) { return g_err; }

}  // extern "C"
