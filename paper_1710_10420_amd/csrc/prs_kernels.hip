// prs_kernels.hip -- float32 instantiation of the PRS kernels (the device
// templates are in prs_device.h), the record reduction, the batched-ensemble
// kernels and the host-side dispatch by precision.

#include <mutex>

#include "prs_device.h"

namespace prs {

namespace {

// Adds `count` wave partials into one record, with one wave, in a fixed
// order: lane l sums partials l, l+64, l+128, ... and the 64 lane sums are
// combined by a fixed butterfly.  Every path that produces a record (single
// run, standalone diagnostics, batched ensemble) calls this function, so a
// record depends only on the partials, never on which kernel reduced them.
__device__ __forceinline__ void finalize_wave(const WavePartial* __restrict__ parts, int64_t count,
                                              prs_stats* __restrict__ rec, int64_t step, double eta,
                                              double area_scale)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t l0 = 0, l1 = 0, l2 = 0, wl = 0, nf = 0;
    double ar = 0.0, ek = 0.0;
#pragma unroll 8
    for (int64_t i = lane; i < count; i += kWave) {
        const WavePartial p = parts[i];
        l0 += p.links[0];
        l1 += p.links[1];
        l2 += p.links[2];
        wl += p.walls;
        nf += p.nonfinite;
        ar += p.area;
        ek += p.ek;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l0 += __shfl_xor(l0, o, kWave);
        l1 += __shfl_xor(l1, o, kWave);
        l2 += __shfl_xor(l2, o, kWave);
        wl += __shfl_xor(wl, o, kWave);
        nf += __shfl_xor(nf, o, kWave);
        ar += __shfl_xor(ar, o, kWave);
        ek += __shfl_xor(ek, o, kWave);
    }
    if (lane == 0) {
        prs_stats r;
        r.step = step;
        r.eta = eta;
        r.links_dir[0] = l0;
        r.links_dir[1] = l1;
        r.links_dir[2] = l2;
        r.links = l0 + l1 + l2;
        r.wall_sites = wl;
        r.nonfinite = nf;
        r.area_density = ar * area_scale;
        r.gv2 = wl ? ek / (double)wl : 0.0;
        *rec = r;
    }
}

__global__ __launch_bounds__(kWave) void k_finalize(const WavePartial* __restrict__ parts,
                                                     int64_t count, prs_stats* __restrict__ rec,
                                                     int64_t step, double eta, double area_scale)
{
    finalize_wave(parts, count, rec, step, eta, area_scale);
}

// Scratch of the allocation-free slab-diagnostics entry point: one record
// slot and the wave partials of one pass, resident on every device the
// library runs on.  Host code never passes this name to a kernel (in host
// code it is only a stand-in for the symbol); static_scratch() hands out the
// device address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Plain device copy of n16 16-byte words (the reference ceiling that pass
// bandwidths are compared with): each 256-lane workgroup moves 16 KiB, four
// independent 16-byte loads per lane in flight before its stores.
__global__ __launch_bounds__(kBlock) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * (4 * kBlock) + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + (int64_t)j * kBlock;
        if (i < n16) v[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + (int64_t)j * kBlock;
        if (i < n16) dst[i] = v[j];
    }
}

// Sum of `count` doubles in a fixed order into *out.
__global__ __launch_bounds__(kBlock) void k_sum_f64(const double* __restrict__ v, int64_t count,
                                                     double* __restrict__ out)
{
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Fills count doubles with 0 (a kernel rather than a memset, so the sequence
// can also live inside a captured graph).
__global__ __launch_bounds__(kBlock) void k_zero_f64(double* __restrict__ v, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) v[i] = 0.0;
}

// ------------------------------------------------------- batched ensemble --
//
// Many independent realisations (different sizes, dimensions, eras, wall
// widths and step counts) advance together.  Each realisation carries a
// table of passes made on the host: a pass advances 1 or 2 steps (two-step
// passes for 2D lattices, never with a recorded state inside), may record the
// diagnostics of its input state, and the last entry is a diagnostics-only
// pass over the final state.  Phase t runs pass t of every realisation that
// has one; each tile runs step_tile or tb_tile, the code of a single run, so
// a realisation's fields and records are bitwise those of the same
// realisation run alone with the same tiling and steps per pass.
//
// Persistent mode: one launch whose workgroups stay resident for the whole
// ensemble; a wave walks the global tile list with stride = number of waves,
// then all workgroups meet at a software grid barrier before the next phase.
// The records of phase t are reduced by one wave per realisation right after
// that barrier.  The barrier's wait is bounded: if it does not complete
// within the time limit (workgroups not co-resident), an error flag is raised
// and every workgroup leaves, so the kernel always finishes.

struct BatchDesc {
    StepArgs A;              // geometry, tiling and constant coefficients
    float* phi[2];           // phase t reads phi[t & 1]
    float* pi_alt;           // second phi_dot buffer for two-step passes (2D)
    const float2* coef;      // (a_n, b_n) for n = 0 .. nsteps-1
    const int4* passes;      // (first step, steps (0: diagnostics only), record or -1, phi_dot in pi_alt)
    WavePartial* part[2];    // alternate record partial buffers
    prs_stats* recs;
    int64_t npasses;         // including the final diagnostics-only pass
    int64_t tile_base;       // first global tile of this realisation
    int64_t tiles_max;       // tiles reserved per phase (the larger pass kind)
    int64_t tiles_multi;     // tiles of a two-step pass (2D)
    double eta0, deta, area_scale;
    int32_t ndim, vec, ty, pad;
};

struct BatchCtl {
    unsigned int arrive;
    unsigned int gen;
    int err;
    int pad;
};

__device__ __forceinline__ int find_real(const BatchDesc* __restrict__ D, int nreal, int64_t tile)
{
    int lo = 0, hi = nreal - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (D[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D, int VEC, int TY>
__device__ __forceinline__ void tile_mode(const StepArgs& A, int64_t tile, bool update, bool diag)
{
    if (update && diag) step_tile<D, VEC, TY, true, true>(A, tile);
    else if (update) step_tile<D, VEC, TY, true, false>(A, tile);
    else step_tile<D, VEC, TY, false, true>(A, tile);
}

// Tilings available inside the batched kernels (every instance is inlined
// into them, so the set is kept small to bound register pressure).
__device__ __forceinline__ void dispatch_tile(int ndim, int vec, const StepArgs& A, int64_t tile,
                                              bool update, bool diag)
{
    if (ndim == 2) {
        if (vec == 4) tile_mode<2, 4, 1>(A, tile, update, diag);
        else if (vec == 2) tile_mode<2, 2, 1>(A, tile, update, diag);
        else tile_mode<2, 1, 1>(A, tile, update, diag);
    } else {
        if (vec == 4) tile_mode<3, 4, 1>(A, tile, update, diag);
        else if (vec == 2) tile_mode<3, 2, 1>(A, tile, update, diag);
        else tile_mode<3, 1, 1>(A, tile, update, diag);
    }
}

__device__ __forceinline__ void dispatch_pair(int vec, const TBArgs<2>& A, int64_t tile, bool diag)
{
    if (vec == 4) {
        if (diag) tb_tile<4, 2, true>(A, tile);
        else tb_tile<4, 2, false>(A, tile);
    } else if (vec == 2) {
        if (diag) tb_tile<2, 2, true>(A, tile);
        else tb_tile<2, 2, false>(A, tile);
    } else {
        if (diag) tb_tile<1, 2, true>(A, tile);
        else tb_tile<1, 2, false>(A, tile);
    }
}

// Work of global tile i in phase t.
__device__ __forceinline__ void batch_tile(const BatchDesc* __restrict__ Dd, int nreal, int64_t i,
                                           int64_t t)
{
    const BatchDesc& d = Dd[find_real(Dd, nreal, i)];
    if (t >= d.npasses) return;
    const int4 ps = d.passes[t];
    const int64_t local = i - d.tile_base;
    const bool diag = ps.z >= 0;
    const float* pin = ps.w ? d.pi_alt : d.A.pi_out;
    if (ps.y == 2) {
        if (local >= d.tiles_multi) return;
        TBArgs<2> A;
        A.phi_in = d.phi[t & 1];
        A.phi_out = d.phi[(t + 1) & 1];
        A.pi_in = pin;
        A.pi_out = ps.w ? d.A.pi_out : d.pi_alt;
        A.partials = diag ? d.part[ps.z & 1] : nullptr;
        A.nx = d.A.nx;
        A.ny = d.A.M;
        A.tiles_x = (d.A.nx + tb_owned_width_d(d.vec, 2) - 1) / tb_owned_width_d(d.vec, 2);
        A.ntiles = d.tiles_multi;
        A.rows = d.A.rows;
        A.k[0] = d.A.k;
        A.k[1] = d.A.k;
        const float2 c0 = d.coef[ps.x], c1 = d.coef[ps.x + 1];
        A.k[0].a = c0.x;
        A.k[0].b = c0.y;
        A.k[1].a = c1.x;
        A.k[1].b = c1.y;
        A.dc = d.A.dc;
        dispatch_pair(d.vec, A, local, diag);
        return;
    }
    if (local >= d.A.ntiles) return;
    StepArgs A = d.A;
    A.phi_in = d.phi[t & 1];
    A.phi_out = d.phi[(t + 1) & 1];
    A.pi = pin;
    A.pi_out = const_cast<float*>(pin);
    const bool update = ps.y == 1;
    if (update) {
        const float2 c = d.coef[ps.x];
        A.k.a = c.x;
        A.k.b = c.y;
    }
    A.partials = diag ? d.part[ps.z & 1] : nullptr;
    dispatch_tile(d.ndim, d.vec, A, local, update, diag);
}

// Records of phase t, one wave per realisation (waves w, w+nw, ...).
__device__ __forceinline__ void batch_records(const BatchDesc* __restrict__ Dd, int nreal, int64_t t,
                                              int64_t wave, int64_t nwaves)
{
    for (int64_t r = wave; r < nreal; r += nwaves) {
        const BatchDesc& d = Dd[r];
        if (t >= d.npasses) continue;
        const int4 ps = d.passes[t];
        if (ps.z < 0) continue;
        const int64_t count = ps.y == 2 ? d.tiles_multi : d.A.ntiles;
        finalize_wave(d.part[ps.z & 1], count, d.recs + ps.z, ps.x, d.eta0 + (double)ps.x * d.deta,
                      d.area_scale);
    }
}

// Grid-wide barrier for a resident grid.  Arrivals count up monotonically;
// the last arrival of generation g publishes g+1.  Release/acquire fences at
// agent scope make every field written before the barrier visible to every
// XCD after it.  Returns false (and raises ctl->err) when the wait exceeds
// `timeout` wall-clock ticks or another workgroup has already failed.
__device__ __forceinline__ bool grid_barrier(BatchCtl* ctl, unsigned nblocks, unsigned gen,
                                             uint64_t timeout)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const unsigned prev =
            __hip_atomic_fetch_add(&ctl->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev + 1u == (gen + 1u) * nblocks) {
            __hip_atomic_store(&ctl->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <= gen) {
                if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > timeout) {
                    __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ __launch_bounds__(kBlock) void k_batch_persistent(const BatchDesc* __restrict__ Dd,
                                                              int nreal, int64_t total_tiles,
                                                              int64_t tmax, BatchCtl* ctl,
                                                              uint64_t timeout)
{
    const int64_t wave = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    unsigned gen = 0;
    for (int64_t t = 0; t <= tmax + 1; ++t) {
        if (t > 0) batch_records(Dd, nreal, t - 1, wave, nwaves);
        if (t > tmax) break;
        for (int64_t i = wave; i < total_tiles; i += nwaves) batch_tile(Dd, nreal, i, t);
        if (!grid_barrier(ctl, gridDim.x, gen, timeout)) return;
        ++gen;
    }
}

// Fallback without a resident grid: one launch per phase over all tiles,
// then one launch for that phase's records.
__global__ __launch_bounds__(kBlock) void k_batch_step(const BatchDesc* __restrict__ Dd, int nreal,
                                                        int64_t total_tiles, int64_t t)
{
    const int64_t i = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (i >= total_tiles) return;
    batch_tile(Dd, nreal, i, t);
}

__global__ __launch_bounds__(kBlock) void k_batch_records(const BatchDesc* __restrict__ Dd, int nreal,
                                                           int64_t t)
{
    const int64_t wave = uniform64((int64_t)blockIdx.x * kWavesPerBlock + wave_in_block());
    batch_records(Dd, nreal, t, wave, (int64_t)gridDim.x * kWavesPerBlock);
}

__global__ __launch_bounds__(kBlock) void k_zero_f32(float* __restrict__ v, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) v[i] = 0.0f;
}

__global__ void k_batch_reset(BatchCtl* ctl)
{
    if (threadIdx.x == 0) {
        ctl->arrive = 0u;
        ctl->gen = 0u;
        ctl->err = 0;
        ctl->pad = 0;
    }
}


}  // namespace

Geometry geometry_of(const prs_params& p)
{
    Geometry g;
    g.ndim = p.ndim;
    g.f64 = p.precision == PRS_F64 ? 1 : 0;
    g.nx = p.n[0];
    if (p.ndim == 2) {
        g.Q = 1;
        g.M = p.n[1];
    } else {
        g.Q = p.n[1];
        g.M = p.n[2];
    }
    return g;
}

TileCounts tile_counts(const Geometry& g, const Tiling& t)
{
    TileCounts c;
    c.tiles_x = (g.nx + (int64_t)kWave * t.vec - 1) / ((int64_t)kWave * t.vec);
    c.tiles_q = (g.Q + step_ty(t.ty) - 1) / step_ty(t.ty);
    c.tiles_s = (g.M + t.rows - 1) / t.rows;
    c.ntiles = c.tiles_x * c.tiles_q * c.tiles_s;
    return c;
}

bool tiling_supported(const Geometry& g, const Tiling& t)
{
    if (t.vec != 1 && t.vec != 2 && t.vec != 4) return false;
    if (g.f64 && t.vec == 4) return false;          // 16 bytes per lane at most
    if (g.nx % t.vec != 0) return false;
    if (t.rows < 1 || t.rows > 4096) return false;
    if (g.ndim == 2) return t.ty == 1;
    return t.ty == 1 || t.ty == 2 || t.ty == 4 || tb3l_tiling(t.ty);
}

// ---- float32 instantiations ----

hipError_t launch_step_f32(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                           void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s)
{
    return launch_step_r<float>(g, t, phi_in, phi_out, pi, pi_out, k, update, diag, partials, dc, s);
}

hipError_t launch_tb_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s)
{
    if (g.ndim == 3) return launch_tb3d_r<float>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
    return launch_tb2d_r<float>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
}

hipError_t launch_tb_slab_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                              const void* pi_in, void* pi_out, const StepCoef64* k, bool diag,
                              WavePartial* partials, const DiagCoef& dc, hipStream_t s)
{
    if (g.ndim == 2)
        return launch_tb2d_r<float>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, T);
    return launch_tb3d_r<float>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, T);
}

hipError_t launch_adjoint_f32(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                              const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s)
{
    return launch_adjoint_r<float>(g, t, w_in, w_out, mu, phi_n, gacc, c, s);
}

hipError_t launch_adj_seed_f32(const void* phi, int64_t count, double kc, double deta, void* mu, void* w,
                               double* partial, int nblocks, hipStream_t s)
{
    return launch_adj_seed_r<float>(phi, count, kc, deta, mu, w, partial, nblocks, s);
}

hipError_t launch_tb_all_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                             const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    return launch_tb_all_r<float>(T, g, t, phi_in, phi_lv, pi_in, pi_out, k, s);
}

hipError_t launch_tba_f32(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                          const void* mu_in, void* mu_out, const void* const* phi, double* gacc,
                          const AdjCoef64* c, hipStream_t s)
{
    return launch_tba_r<float>(T, g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);
}

hipError_t launch_tb_mid_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                             const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                             hipStream_t s)
{
    return launch_tb_mid_r<float>(T, g, t, phi_in, phi_out, pi_in, pi_out, phi_mid, pi_mid, k, s);
}

hipError_t launch_tbf_f32(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                          const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                          const StepCoef64* k, const AdjCoef64* c, hipStream_t s)
{
    return launch_tbf_r<float>(T, g, t, phi_s, pi_s, w_in, w_out, mu_in, mu_out, gacc, k, c, s);
}

hipError_t launch_fill_f32(void* phi, int64_t count, uint64_t seed, hipStream_t s)
{
    return launch_fill_r<float>(phi, count, seed, s);
}

// ---- dispatch by precision ----

hipError_t launch_step(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                       void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                       const DiagCoef& dc, hipStream_t s)
{
    if (!tiling_supported(g, t)) return hipErrorInvalidValue;
    return g.f64 ? launch_step_f64(g, t, phi_in, phi_out, pi, pi_out, k, update, diag, partials, dc, s)
                 : launch_step_f32(g, t, phi_in, phi_out, pi, pi_out, k, update, diag, partials, dc, s);
}

hipError_t launch_tb(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                     const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                     const DiagCoef& dc, hipStream_t s)
{
    if (!tb_pass_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tb_f64(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s)
                 : launch_tb_f32(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
}

hipError_t launch_tb_slab(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                          const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                          const DiagCoef& dc, hipStream_t s)
{
    if (!tb_pass_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tb_slab_f64(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s)
                 : launch_tb_slab_f32(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
}

hipError_t launch_adjoint(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                          const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s)
{
    if (!tiling_supported(g, t)) return hipErrorInvalidValue;
    return g.f64 ? launch_adjoint_f64(g, t, w_in, w_out, mu, phi_n, gacc, c, s)
                 : launch_adjoint_f32(g, t, w_in, w_out, mu, phi_n, gacc, c, s);
}

hipError_t launch_adj_seed(const Geometry& g, const void* phi, int64_t count, double kc, double deta, void* mu,
                           void* w, double* partial, int nblocks, hipStream_t s)
{
    return g.f64 ? launch_adj_seed_f64(phi, count, kc, deta, mu, w, partial, nblocks, s)
                 : launch_adj_seed_f32(phi, count, kc, deta, mu, w, partial, nblocks, s);
}

bool tba_supported(const Geometry& g, const Tiling& t, int T)
{
    if (!tb_supported(g) || !tiling_supported(g, t)) return false;
    if (g.ndim == 3 && tb3l_tiling(t.ty)) return false;
    if (g.ndim == 3) {
        const int TY = tb3_rows(t.ty);
        return g.f64 ? tba3_combo_ok<double>(t.vec, T, TY) : tba3_combo_ok<float>(t.vec, T, TY);
    }
    if (t.ty != 1) return false;
    return g.f64 ? tba_combo_ok<double>(t.vec, T) : tba_combo_ok<float>(t.vec, T);
}

bool tb_all_supported(const Geometry& g, const Tiling& t, int T)
{
    if (g.ndim == 3) return tb_pass_supported(g, t, T);
    if (!tb_supported(g) || !tiling_supported(g, t) || t.ty != 1) return false;
    return g.f64 ? tball_combo_ok<double>(t.vec, T) : tball_combo_ok<float>(t.vec, T);
}

hipError_t launch_tb_all(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                         const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    if (!tb_all_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tb_all_f64(T, g, t, phi_in, phi_lv, pi_in, pi_out, k, s)
                 : launch_tb_all_f32(T, g, t, phi_in, phi_lv, pi_in, pi_out, k, s);
}

hipError_t launch_tba(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out, const void* mu_in,
                      void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c, hipStream_t s)
{
    if (!tba_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tba_f64(T, g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s)
                 : launch_tba_f32(T, g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);
}

bool tb_mid_supported(const Geometry& g, const Tiling& t, int T)
{
    if (g.ndim != 2 || !tb_supported(g) || !tiling_supported(g, t) || t.ty != 1) return false;
    return g.f64 ? tbmid_combo_ok<double>(t.vec, T) : tbmid_combo_ok<float>(t.vec, T);
}

hipError_t launch_tb_mid(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                         hipStream_t s)
{
    if (!tb_mid_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tb_mid_f64(T, g, t, phi_in, phi_out, pi_in, pi_out, phi_mid, pi_mid, k, s)
                 : launch_tb_mid_f32(T, g, t, phi_in, phi_out, pi_in, pi_out, phi_mid, pi_mid, k, s);
}

bool tbf_supported(const Geometry& g, const Tiling& t, int T)
{
    if (g.ndim != 2 || !tb_supported(g) || !tiling_supported(g, t) || t.ty != 1) return false;
    return g.f64 ? tbf_combo_ok<double>(t.vec, T) : tbf_combo_ok<float>(t.vec, T);
}

int64_t tbf_tiles(const Geometry& g, const Tiling& t, int T)
{
    const int64_t W = (int64_t)(kWave - 2 * tbf_halo(t.vec, T)) * t.vec;
    return ((g.nx + W - 1) / W) * ((g.M + t.rows - 1) / t.rows);
}

hipError_t launch_tbf(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                      const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                      const StepCoef64* k, const AdjCoef64* c, hipStream_t s)
{
    if (!tbf_supported(g, t, T)) return hipErrorInvalidValue;
    return g.f64 ? launch_tbf_f64(T, g, t, phi_s, pi_s, w_in, w_out, mu_in, mu_out, gacc, k, c, s)
                 : launch_tbf_f32(T, g, t, phi_s, pi_s, w_in, w_out, mu_in, mu_out, gacc, k, c, s);
}

hipError_t launch_fill_uniform(void* phi, int64_t count, uint64_t seed, bool f64, hipStream_t s)
{
    return f64 ? launch_fill_f64(phi, count, seed, s) : launch_fill_f32(phi, count, seed, s);
}

hipError_t launch_finalize(const WavePartial* partials, int64_t count, prs_stats* rec,
                           int64_t step, double eta, double area_scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kWave), 0, s, partials, count, rec, step, eta,
                       area_scale);
    return hipGetLastError();
}

hipError_t static_scratch(void** ptr, size_t* bytes)
{
    // the device address of `scratch` on each device, looked up once per
    // device with that device current (each device holds its own copy)
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s)
{
    if (n16 <= 0) return hipSuccess;
    const int64_t blocks = (n16 + 4 * kBlock - 1) / (4 * kBlock);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kBlock), 0, s, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_sum_f64(const double* v, int64_t count, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kBlock), 0, s, v, count, out);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* v, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)blocks), dim3(kBlock), 0, s, v, count);
    return hipGetLastError();
}

// ---- batched ensemble launchers ----

size_t batch_desc_bytes() { return sizeof(BatchDesc); }

void batch_fill_desc(void* out, const Geometry& g, const Tiling& t, float* phi0, float* phi1, float* pi,
                     float* pi_alt, const float2* coef, const void* passes, int64_t npasses,
                     WavePartial* part0, WavePartial* part1, prs_stats* recs, int64_t tile_base,
                     double eta0, double deta, double area_scale, const StepCoef& k, const DiagCoef& dc)
{
    const TileCounts c = tile_counts(g, t);
    BatchDesc d;
    d.A.phi_in = nullptr;
    d.A.phi_out = nullptr;
    d.A.pi = pi;
    d.A.pi_out = pi;
    d.A.partials = nullptr;
    d.A.nx = g.nx;
    d.A.Q = g.Q;
    d.A.M = g.M;
    d.A.tiles_x = c.tiles_x;
    d.A.tiles_q = c.tiles_q;
    d.A.ntiles = c.ntiles;
    d.A.rows = t.rows;
    d.A.k = k;
    d.A.dc = dc;
    d.phi[0] = phi0;
    d.phi[1] = phi1;
    d.pi_alt = pi_alt;
    d.coef = coef;
    d.passes = static_cast<const int4*>(passes);
    d.part[0] = part0;
    d.part[1] = part1;
    d.recs = recs;
    d.npasses = npasses;
    d.tile_base = tile_base;
    d.tiles_multi = g.ndim == 2 ? tb_tiles(g, t, 2) : 0;
    d.tiles_max = std::max<int64_t>(c.ntiles, d.tiles_multi);
    d.eta0 = eta0;
    d.deta = deta;
    d.area_scale = area_scale;
    d.ndim = g.ndim;
    d.vec = t.vec;
    d.ty = t.ty;
    d.pad = 0;
    *static_cast<BatchDesc*>(out) = d;
}

int64_t batch_tiles_max(const Geometry& g, const Tiling& t)
{
    const int64_t a = tile_counts(g, t).ntiles;
    return g.ndim == 2 ? std::max<int64_t>(a, tb_tiles(g, t, 2)) : a;
}

bool batch_tiling_supported(const Geometry& g, const Tiling& t)
{
    return tiling_supported(g, t) && t.ty == 1;
}

hipError_t batch_max_blocks(int* blocks)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_persistent, kBlock, 0);
    if (e != hipSuccess) return e;
    *blocks = cus * per;
    return hipSuccess;
}

hipError_t batch_clock_rate_khz(int* khz)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev);
}

hipError_t launch_batch_reset(void* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kWave), 0, s, static_cast<BatchCtl*>(ctl));
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const void* descs, int nreal, int64_t total_tiles, int64_t tmax,
                                   void* ctl, uint64_t timeout, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_persistent, dim3(blocks), dim3(kBlock), 0, s,
                       static_cast<const BatchDesc*>(descs), nreal, total_tiles, tmax,
                       static_cast<BatchCtl*>(ctl), timeout);
    return hipGetLastError();
}

hipError_t launch_batch_step(const void* descs, int nreal, int64_t total_tiles, int64_t t, hipStream_t s)
{
    const int64_t blocks = (total_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_batch_step, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       static_cast<const BatchDesc*>(descs), nreal, total_tiles, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int rb = (nreal + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_batch_records, dim3(rb), dim3(kBlock), 0, s, static_cast<const BatchDesc*>(descs),
                       nreal, t);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* v, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(kBlock), 0, s, v, count);
    return hipGetLastError();
}

int batch_ctl_bytes() { return (int)sizeof(BatchCtl); }


int64_t tb_owned_width(int vec, int T)
{
    const int H = (T + vec - 1) / vec;
    return (int64_t)(kWave - 2 * H) * vec;
}


bool tb_supported(const Geometry& g)
{
    if (g.ndim == 2) return g.nx <= ((int64_t)1 << 28);
    return g.nx * g.Q * (g.f64 ? 8 : 4) < ((int64_t)1 << 31);
}

bool tb_steps_supported(const Geometry& g, int T)
{
    if (!tb_supported(g)) return false;
    if (g.ndim == 3) return T == 2 || T == 3 || T == 4;
    return T == 2 || T == 3 || T == 4 || T == 6 || T == 8;
}

bool tb_pass_supported(const Geometry& g, const Tiling& t, int T)
{
    if (!tb_steps_supported(g, T) || !tiling_supported(g, t)) return false;
    if (g.ndim == 2) return t.ty == 1 && (g.f64 ? tb2_combo_ok<double>(t.vec, T) : tb2_combo_ok<float>(t.vec, T));
    if (tb3l_tiling(t.ty)) {
        const int rw = tb3l_rows_per_wave(t.ty), nw = tb3l_waves(t.ty);
        return g.f64 ? tb3l_combo_ok<double>(t.vec, T, rw, nw) : tb3l_combo_ok<float>(t.vec, T, rw, nw);
    }
    return g.f64 ? tb3_combo_ok<double>(t.vec, T, tb3_rows(t.ty)) : tb3_combo_ok<float>(t.vec, T, tb3_rows(t.ty));
}

int64_t tb_tiles(const Geometry& g, const Tiling& t, int T)
{
    const int64_t W = tb_owned_width(t.vec, T);
    const int64_t planes = (g.M + t.rows - 1) / t.rows;
    if (g.ndim == 3 && tb3l_tiling(t.ty)) {
        // one partial per wave of every workgroup
        const int nw = tb3l_waves(t.ty);
        const int64_t yown = tb3l_own_rows(nw, tb3l_rows_per_wave(t.ty), T);
        return ((g.nx + W - 1) / W) * ((g.Q + yown - 1) / yown) * planes * nw;
    }
    if (g.ndim == 3) {
        const int64_t TY = tb3_rows(t.ty);
        return ((g.nx + W - 1) / W) * ((g.Q + TY - 1) / TY) * planes;
    }
    return ((g.nx + W - 1) / W) * planes;
}

}  // namespace prs
