// prs_kernels_f64.hip -- float64 instantiation of the PRS kernels (the
// device templates are in prs_device.h).  The paper runs its kernels in
// single and in double precision (Sec. III, Table I); the double kernels are
// the same code with 8-byte fields: 32 B of HBM traffic per site-update,
// lanes of 1 or 2 sites (16 bytes per access at most).

#include "prs_device.h"

namespace prs {

hipError_t launch_step_f64(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                           void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s)
{
    return launch_step_r<double>(g, t, phi_in, phi_out, pi, pi_out, k, update, diag, partials, dc, s);
}

hipError_t launch_tb_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s)
{
    if (g.ndim == 3) return launch_tb3d_r<double>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
    return launch_tb2d_r<double>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s);
}

hipError_t launch_tb_slab_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                              const void* pi_in, void* pi_out, const StepCoef64* k, bool diag,
                              WavePartial* partials, const DiagCoef& dc, hipStream_t s)
{
    if (g.ndim == 2)
        return launch_tb2d_r<double>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, T);
    return launch_tb3d_r<double>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, T);
}

hipError_t launch_adjoint_f64(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                              const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s)
{
    return launch_adjoint_r<double>(g, t, w_in, w_out, mu, phi_n, gacc, c, s);
}

hipError_t launch_adj_seed_f64(const void* phi, int64_t count, double kc, double deta, void* mu, void* w,
                               double* partial, int nblocks, hipStream_t s)
{
    return launch_adj_seed_r<double>(phi, count, kc, deta, mu, w, partial, nblocks, s);
}

hipError_t launch_tb_all_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                             const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    return launch_tb_all_r<double>(T, g, t, phi_in, phi_lv, pi_in, pi_out, k, s);
}

hipError_t launch_tba_f64(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                          const void* mu_in, void* mu_out, const void* const* phi, double* gacc,
                          const AdjCoef64* c, hipStream_t s)
{
    return launch_tba_r<double>(T, g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);
}

hipError_t launch_tb_mid_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                             const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                             hipStream_t s)
{
    return launch_tb_mid_r<double>(T, g, t, phi_in, phi_out, pi_in, pi_out, phi_mid, pi_mid, k, s);
}

hipError_t launch_tbf_f64(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                          const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                          const StepCoef64* k, const AdjCoef64* c, hipStream_t s)
{
    return launch_tbf_r<double>(T, g, t, phi_s, pi_s, w_in, w_out, mu_in, mu_out, gacc, k, c, s);
}

hipError_t launch_fill_f64(void* phi, int64_t count, uint64_t seed, hipStream_t s)
{
    return launch_fill_r<double>(phi, count, seed, s);
}

}  // namespace prs
