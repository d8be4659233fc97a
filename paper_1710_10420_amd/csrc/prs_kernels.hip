// prs_kernels.hip -- float32 instantiation of the PRS kernels (the device
// templates are in prs_device.h), the record reduction and the host-side
// dispatch by precision (the batched ensemble's kernel is in prs_ensemble.hip).

#include <mutex>

#include "prs_device.h"

namespace prs {

namespace {

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

__global__ __launch_bounds__(kBlock) void k_zero_f32(float* __restrict__ v, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) v[i] = 0.0f;
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

int64_t tb2_workgroups(const Geometry& g, const Tiling& t, int T)
{
    return (tb_tiles(g, t, T) + kWavesPerBlock - 1) / kWavesPerBlock;
}

int64_t tbf_workgroups(const Geometry& g, const Tiling& t, int T)
{
    return (tbf_tiles(g, t, T) + kWavesPerBlock - 1) / kWavesPerBlock;
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

hipError_t batch_clock_rate_khz(int* khz)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev);
}

hipError_t launch_zero_f32(float* v, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(kBlock), 0, s, v, count);
    return hipGetLastError();
}



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
