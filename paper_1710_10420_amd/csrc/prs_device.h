// prs_device.h -- gfx950 device code of the PRS domain-wall evolution
// (arXiv:1710.10420, Sec. II, Eqs. 3-8), templated on the field precision R
// (float or double; the paper runs both, Sec. III), with the host-side launch
// templates.  Included by the float32 and the float64 kernel files, each of
// which instantiates the kernels of its precision.
//
// One kernel does a whole step: the Laplacian (Eq. 3), the damped kick
// (Eqs. 4, 6) and the drift (Eq. 5), and on diagnostic steps the wall area
// (Eq. 7) and velocity (Eq. 8) sums of the step's input state.  The paper ran
// these as separate kernels through global memory and named fusing them as
// the next step; here each field value crosses HBM once per step: phi^n and
// phi_dot are read once, phi^{n+1} and phi_dot written once (16 B per site
// in float32, 32 B in float64).
//
// Work decomposition.  A wave (64 lanes) owns a tile of
//   64*VEC sites along x  x  TY rows along the middle axis (3D only)
// and marches along the slowest axis (y in 2D, z in 3D) through `rows`
// planes.  The three planes s-1, s, s+1 it needs stay in registers and the
// plane s+2 is already in flight while s is computed, so every phi value is
// loaded from HBM once per tile.  x-neighbours come from the adjacent lane
// (wave-wide DPP shifts); only the two wave-edge lanes load a halo scalar.
// In 3D the rows above and below the tile are loaded per plane and are
// served by L2, because the waves of a workgroup hold consecutive rows and
// consecutive workgroups of one XCD hold consecutive tiles (xcd_remap).
// Waves are independent: no LDS, no barriers.
//
// Arithmetic.  Every site runs the same inline sequence (explicit fused
// multiply-adds, -ffp-contract=off), so results are bitwise independent of
// the tiling, of the lane a site lands in and of the batch it runs in.
// Neighbour sums are grouped as (phi_- + phi_+) pairs, which makes x -> -x
// reflections and phi -> -phi exact symmetries of the update as well.
//
// Diagnostics.  Sign bits s = (phi >= 0) give the crossing links; counts are
// per-lane 32-bit, reduced per wave with butterfly shuffles; the Eq. (7)
// weight and the Eq. (8) ratio are evaluated in FP64 only at sites that
// touch a wall.  Each wave writes one WavePartial; a single-wave finalize
// kernel adds them in index order, so the record is deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <utility>

#include "prs_internal.h"

namespace prs {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8).  Give each XCD a contiguous range of logical blocks so that
// tiles that share halo rows run on the same XCD, close in time, and their
// shared rows hit that XCD's L2.  Bijective for any grid size.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    int64_t xcd = b % kXcds, k = b / kXcds;
    int64_t per = nb / kXcds, rem = nb % kXcds;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// 3D tilings with ty 8, 16, 32 or 64 select the LDS-staged multi-step pass
// (eight waves of 2 or 4 rows for ty 8, 16; sixteen waves of 2 or 4 rows for
// ty 32, 64); their single steps and reverse steps run the one-row kernels
// of ty 1 (whose registers stay low enough for the ensemble kernel).
__host__ __device__ __forceinline__ bool tb3l_tiling(int ty) { return ty == 8 || ty == 16 || ty == 32 || ty == 64; }

__host__ __device__ __forceinline__ int step_ty(int ty) { return ty > 4 ? 1 : ty; }

// Index of this wave within its workgroup, as a wave-uniform (scalar) value:
// the compiler cannot prove threadIdx.x / 64 uniform on its own, and every
// address derived from it would otherwise be computed per lane.
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Makes a wave-uniform 64-bit value visibly uniform to the compiler.
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t wrap(int64_t v, int64_t n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Fused multiply-add in the field precision (one rounding).
__device__ __forceinline__ float fmar(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return fma(a, b, c); }

template <int VEC, typename R>
__device__ __forceinline__ void load_vec(const R* p, R (&v)[VEC])
{
    static_assert(VEC * sizeof(R) <= 16, "at most 16 bytes per lane and access");
    if constexpr (VEC == 4) {
        float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (VEC == 2 && sizeof(R) == 4) {
        float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x; v[1] = t.y;
    } else if constexpr (VEC == 2) {
        double2 t = *reinterpret_cast<const double2*>(p);
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = *p;
    }
}

template <int VEC, typename R>
__device__ __forceinline__ void store_vec(R* p, const R (&v)[VEC])
{
    static_assert(VEC * sizeof(R) <= 16, "at most 16 bytes per lane and access");
    if constexpr (VEC == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (VEC == 2 && sizeof(R) == 4) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else if constexpr (VEC == 2) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    } else {
        *p = v[0];
    }
}

// Sum of the 2D nearest neighbours of a site (the non-central part of Eq. 3).
template <typename R>
__device__ __forceinline__ R nsum2(R xm, R xp, R ym, R yp)
{
    return (xm + xp) + (ym + yp);
}

template <typename R>
__device__ __forceinline__ R nsum3(R xm, R xp, R ym, R yp, R zm, R zp)
{
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// Eqs. (3)-(5) with the FP64-derived coefficients of StepCoefT, from the
// neighbour sum s of a site in D dimensions:
//   pi' = a pi + b (Lap phi - V'(phi)),  Lap phi = (s - 2D phi)/dx^2,
//   V'(phi) = F phi (kc phi^2 - 1).
// In 2D it is evaluated as a pi + (b/dx^2) s - phi (4 b/dx^2 + (b F)(kc phi^2 - 1)):
// the central term of the Laplacian joins the force, six operations per site
// after the neighbour sum; 4 b/dx^2 is exact, so a homogeneous vacuum
// (s = 4 phi, phi^2 = 1) gets exactly zero force.  In 3D 6 b/dx^2 would be
// rounded and a vacuum would drift, so the Laplacian is formed first,
// (s - 6 phi)/dx^2, and the kick is a pi + (b Lap phi - (b F) phi (kc phi^2 - 1)).
// b/dx^2, 4 b/dx^2 and b F are wave-uniform products per launch (hoisted out
// of the march).  UNIT (dx = 1, phi0 = 1) drops the exact multiplications by 1.
template <int D, bool UNIT = false, typename R>
__device__ __forceinline__ void kick_drift(R c, R s, R pi, const StepCoefT<R>& k, R& pi_new, R& phi_new)
{
    const R ck = UNIT ? c : c * k.kc;
    const R q = fmar(ck, c, R(-1));
    R v;
    if constexpr (D == 2) {
        const R bl = UNIT ? k.b : k.b * k.inv_dx2;
        const R t = fmar(k.b * k.F, q, R(4) * bl);   // 4 b/dx^2 + (b F)(kc phi^2 - 1)
        v = fmar(bl, s, -(c * t));                    // b (Lap phi - V'(phi))
    } else {
        const R r = fmar(R(-2 * D), c, s);
        const R lap = UNIT ? r : r * k.inv_dx2;
        v = fmar(-((k.b * k.F) * c), q, k.b * lap);   // b (Lap phi - V'(phi))
    }
    pi_new = fmar(k.a, pi, v);                         // Eq. (4)
    phi_new = fmar(k.deta, pi_new, c);                 // Eq. (5)
}

// One reverse step at a site (the transpose of Eqs. 3-5 for the adjoint
// pair w = adjoint of phi_dot, mu = adjoint of phi), from the neighbour sum s
// of w and phi = phi^n at the site:
//   mu' = mu + b (Lap w - V''(phi) w),  w' = a w + cw mu',
//   V''(phi) = F (3 kc phi^2 - 1),
// with Lap w - V''(phi) w = s/dx^2 - w (3F (kc phi^2 - 1) + 2F + 2D/dx^2): the
// central term of the Laplacian joins V'', and kc phi^2 - 1 is shared with the
// dL/dV0 term w phi (kc phi^2 - 1), which is returned.  2F + 2D/dx^2 is one
// wave-uniform constant per launch.
template <int D, bool UNIT = false, typename R>
__device__ __forceinline__ R adj_site(R w, R s, R mu, R phi, R a, R b, R cw, R F, R kc, R inv_dx2, R& w_new,
                                      R& mu_new)
{
    const R pk = UNIT ? phi : phi * kc;
    const R q = fmar(pk, phi, R(-1));                                      // kc phi^2 - 1
    const R c1 = fmar(R(2), F, UNIT ? R(2 * D) : R(2 * D) * inv_dx2);      // 2F + 2D/dx^2
    const R t = fmar(R(3) * F, q, c1);
    const R x = fmar(-w, t, UNIT ? s : s * inv_dx2);                       // Lap w - V''(phi) w
    mu_new = fmar(b, x, mu);
    w_new = fmar(cw, mu_new, a * w);
    return w * (phi * q);
}

// Value held by the lane on the left (lane - 1) / right (lane + 1) of this
// one, by a wave-wide DPP shift.  The end lane (lane 0 / lane 63) has no
// source and reads 0; every caller either replaces that value (halo loads of
// the single-step march) or never stores the end lanes' results (overlapped
// tiles of the multi-step passes).  Without an "old" operand the compiler can
// fold the shift into the instruction that consumes it.
__device__ __forceinline__ float from_left_lane(float v)
{
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(b, 0x138, 0xF, 0xF, true));
}

__device__ __forceinline__ float from_right_lane(float v)
{
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(b, 0x130, 0xF, 0xF, true));
}

// The same shifts for a double: both 32-bit halves move together.
__device__ __forceinline__ double from_left_lane(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
    const uint32_t l = (uint32_t)__builtin_amdgcn_mov_dpp(lo, 0x138, 0xF, 0xF, true);
    const uint32_t h = (uint32_t)__builtin_amdgcn_mov_dpp(hi, 0x138, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)h << 32) | l);
}

__device__ __forceinline__ double from_right_lane(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
    const uint32_t l = (uint32_t)__builtin_amdgcn_mov_dpp(lo, 0x130, 0xF, 0xF, true);
    const uint32_t h = (uint32_t)__builtin_amdgcn_mov_dpp(hi, 0x130, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)h << 32) | l);
}

struct DiagAcc {
    uint32_t links[3];
    uint32_t walls;
    uint32_t nonfinite;
    double area;
    double ek;
};

// Eqs. (7)-(8) contribution of one site: forward links along each axis,
// the wall flag from forward and backward links, the area weight
// |g| / sum|g_d| from centred differences (the 1/(2 dx) factor cancels), and
// (1/2) phi_dot^2 / V at wall sites.
template <int D, typename R>
__device__ __forceinline__ void site_diag(R c, R pi, const R (&nm)[D], const R (&np)[D], const DiagCoef& dc,
                                          DiagAcc& a)
{
    const bool sc = c >= R(0);
    int cross = 0;
    bool wall = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const bool fwd = sc != (np[d] >= R(0));
        const bool bwd = sc != (nm[d] >= R(0));
        a.links[d] += fwd ? 1u : 0u;
        cross += fwd ? 1 : 0;
        wall = wall || fwd || bwd;
    }
    if (!(__builtin_isfinite(c) && __builtin_isfinite(pi))) a.nonfinite += 1u;
    a.walls += wall ? 1u : 0u;
    // The FP64 terms are evaluated only by waves that have a crossing link
    // (a wall site) among their lanes: walls are sparse once the network has
    // coarsened, and without the wave-uniform test the compiler evaluates
    // both square root and divisions on every site.
    if (__builtin_amdgcn_ballot_w64(cross != 0)) {
        if (cross) {
            double gsq = 0.0, gabs = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double h = (double)np[d] - (double)nm[d];
                gsq += h * h;
                gabs += fabs(h);
            }
            double w = gabs > 0.0 ? sqrt(gsq) / gabs : 1.0;
            a.area += (double)cross * w;
        }
    }
    if (__builtin_amdgcn_ballot_w64(wall)) {
        if (wall) {
            double cd = (double)c;
            double q = cd * cd * dc.kc - 1.0;
            double V = dc.V0 * q * q;
            if (V > 0.0) {
                double pd = (double)pi;
                a.ek += 0.5 * pd * pd / V;
            }
        }
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

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

template <typename R>
struct StepArgsT {
    const R* phi_in;
    R* phi_out;
    const R* pi;           // phi_dot^{n-1/2} (read)
    R* pi_out;             // phi_dot^{n+1/2} (written; may equal pi)
    WavePartial* partials;
    int64_t nx, Q, M;
    int64_t tiles_x, tiles_q, ntiles;
    int64_t rows;
    StepCoefT<R> k;
    DiagCoef dc;
};
using StepArgs = StepArgsT<float>;

// One plane of a wave's tile: TY rows of VEC sites per lane, the two x-halo
// scalars (used by lane 0 / the last active lane) and, in 3D, the rows just
// above and below the tile.
template <int VEC, int TY, typename R>
struct Plane {
    R v[TY][VEC];
    R hl[TY];
    R hr[TY];
    R lo[VEC];
    R hi[VEC];
};

// Everything a wave needs to walk its tile, computed once.  In-plane offsets
// are unsigned 32-bit (a plane holds fewer than 2^31 sites), plane bases are
// wave-uniform 64-bit pointers, so the march needs no division and loads use
// the scalar-base + vector-offset form.
template <int TY>
struct TileSetup {
    uint32_t x0, xl, xr;     // this lane's first site and its x-halo sites
    bool active, need_left, need_right;
    uint32_t off[TY];        // (q0 + t) * nx + x0
    uint32_t offl[TY];       // (q0 + t) * nx + xl
    uint32_t offr[TY];       // (q0 + t) * nx + xr
    uint32_t lo, hi;         // rows above / below the tile (3D), + x0
    int nvalid;              // rows of the tile inside the lattice
    int64_t s0, s1;          // marching range
    int64_t M, pstride;
};

// Plane index wrapped into [0, M) for v in [-1, 2M]: no division.
__device__ __forceinline__ int64_t wrap_plane(int64_t v, int64_t M)
{
    if (v < 0) v += M;
    if (v >= M) v -= M;
    if (v >= M) v -= M;
    return v;
}

template <int VEC, int TY>
__device__ __forceinline__ TileSetup<TY> tile_setup(int64_t nx64, int64_t Q64, int64_t M,
                                                    int64_t tiles_x, int64_t tiles_q, int64_t rows,
                                                    int64_t tile)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tq = tl % (uint32_t)tiles_q;
    const uint32_t rest = tl / (uint32_t)tiles_q;
    const uint32_t tx = rest % (uint32_t)tiles_x;
    const uint32_t ts = rest / (uint32_t)tiles_x;
    const uint32_t nx = (uint32_t)nx64, Q = (uint32_t)Q64;
    TileSetup<TY> S;
    S.x0 = tx * (kWave * VEC) + lane * VEC;
    S.active = S.x0 < nx;
    S.need_left = S.active && lane == 0;
    S.need_right = S.active && (lane == kWave - 1 || S.x0 + VEC >= nx);
    S.xl = S.x0 == 0 ? nx - 1 : S.x0 - 1;
    S.xr = S.x0 + VEC >= nx ? 0 : S.x0 + VEC;
    const uint32_t q0 = tq * TY;
    S.nvalid = (int)((Q - q0) < (uint32_t)TY ? (Q - q0) : (uint32_t)TY);
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        const uint32_t r = (q0 + t) * nx;
        S.off[t] = r + S.x0;
        S.offl[t] = r + S.xl;
        S.offr[t] = r + S.xr;
    }
    uint32_t lo = q0 == 0 ? Q - 1 : q0 - 1;
    uint32_t hi = q0 + (uint32_t)S.nvalid;
    while (hi >= Q) hi -= Q;          // Q >= 1; a few iterations at most when Q < TY
    S.lo = lo * nx + S.x0;
    S.hi = hi * nx + S.x0;
    S.s0 = (int64_t)ts * rows;
    S.s1 = (S.s0 + rows) < M ? (S.s0 + rows) : M;
    S.M = M;
    S.pstride = nx64 * Q64;
    return S;
}

template <int D, int VEC, int TY, typename R>
__device__ __forceinline__ void load_plane(const R* __restrict__ f, int64_t s,
                                           const TileSetup<TY>& S, Plane<VEC, TY, R>& P)
{
    const R* base = f + wrap_plane(s, S.M) * S.pstride;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        if (t < S.nvalid) {
            if (S.active) load_vec<VEC>(base + S.off[t], P.v[t]);
            if (S.need_left) P.hl[t] = base[S.offl[t]];
            if (S.need_right) P.hr[t] = base[S.offr[t]];
        }
    }
    if constexpr (D == 3) {
        if (S.active) {
            load_vec<VEC>(base + S.lo, P.lo);
            load_vec<VEC>(base + S.hi, P.hi);
        }
    }
}

// A plane that is only needed for its values along the marching axis (s-1):
// no x-halo scalars, no y-halo rows.
template <int VEC, int TY, typename R>
__device__ __forceinline__ void load_plane_values(const R* __restrict__ f, int64_t s,
                                                  const TileSetup<TY>& S, Plane<VEC, TY, R>& P)
{
    const R* base = f + wrap_plane(s, S.M) * S.pstride;
#pragma unroll
    for (int t = 0; t < TY; ++t)
        if (t < S.nvalid && S.active) load_vec<VEC>(base + S.off[t], P.v[t]);
}

// Point-wise field values of plane s (s inside the lattice) for every row.
template <int VEC, int TY, typename R>
__device__ __forceinline__ void load_point(const R* __restrict__ f, int64_t s,
                                           const TileSetup<TY>& S, R (&v)[TY][VEC])
{
    const R* base = f + s * S.pstride;
#pragma unroll
    for (int t = 0; t < TY; ++t)
        if (t < S.nvalid && S.active) load_vec<VEC>(base + S.off[t], v[t]);
}

template <int VEC, int TY, typename R>
__device__ __forceinline__ void zero_plane(Plane<VEC, TY, R>& P)
{
#pragma unroll
    for (int t = 0; t < TY; ++t) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) P.v[t][j] = R(0);
        P.hl[t] = P.hr[t] = R(0);
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) P.lo[j] = P.hi[j] = R(0);
}

template <int VEC, int TY, typename R>
__device__ __forceinline__ void zero_rows(R (&v)[TY][VEC])
{
#pragma unroll
    for (int t = 0; t < TY; ++t)
#pragma unroll
        for (int j = 0; j < VEC; ++j) v[t][j] = R(0);
}

// x-neighbours of the first and last site of each row of the current plane.
template <int VEC, int TY, typename R>
__device__ __forceinline__ void x_neighbours(const Plane<VEC, TY, R>& P, const TileSetup<TY>& S,
                                             R (&left)[TY], R (&right)[TY])
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        left[t] = from_left_lane(P.v[t][VEC - 1]);
        right[t] = from_right_lane(P.v[t][0]);
        if (lane == 0) left[t] = P.hl[t];
        if (S.need_right) right[t] = P.hr[t];
    }
}

// The 2D neighbours (minus, plus) of site j of row t of the current plane.
template <int D, int VEC, int TY, typename R>
__device__ __forceinline__ void neighbours(const Plane<VEC, TY, R>& Pm, const Plane<VEC, TY, R>& Pc,
                                           const Plane<VEC, TY, R>& Pn, const R (&left)[TY],
                                           const R (&right)[TY], int nvalid, int t, int j,
                                           R (&nm)[D], R (&np)[D])
{
    nm[0] = j > 0 ? Pc.v[t][j > 0 ? j - 1 : 0] : left[t];
    np[0] = j < VEC - 1 ? Pc.v[t][j < VEC - 1 ? j + 1 : j] : right[t];
    if constexpr (D == 3) {
        nm[1] = t > 0 ? Pc.v[t > 0 ? t - 1 : 0][j] : Pc.lo[j];
        np[1] = (t + 1 < nvalid) ? Pc.v[t + 1 < TY ? t + 1 : t][j] : Pc.hi[j];
        nm[2] = Pm.v[t][j];
        np[2] = Pn.v[t][j];
    } else {
        nm[1] = Pm.v[t][j];
        np[1] = Pn.v[t][j];
    }
}

// Plane s of a forward tile: prefetch plane s+2 (and phi_dot of s+1), then
// update plane s from (Pm, Pc, Pn) = planes (s-1, s, s+1).
template <int D, int VEC, int TY, bool UPDATE, bool DIAG, bool UNIT = false, typename R = float>
__device__ __forceinline__ void step_plane(const StepArgsT<R>& A, const TileSetup<TY>& S, int64_t s,
                                           const Plane<VEC, TY, R>& Pm, const Plane<VEC, TY, R>& Pc,
                                           const Plane<VEC, TY, R>& Pn, Plane<VEC, TY, R>& Pnn,
                                           const R (&pic)[TY][VEC], R (&pin)[TY][VEC], DiagAcc& acc)
{
    if (s + 1 < S.s1) {
        load_plane<D, VEC, TY>(A.phi_in, s + 2, S, Pnn);
        load_point<VEC, TY>(A.pi, s + 1, S, pin);
    }
    R left[TY], right[TY];
    x_neighbours<VEC, TY>(Pc, S, left, right);
    R* phi_out = A.phi_out + s * S.pstride;
    R* pi_out = A.pi_out + s * S.pstride;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        if (t >= S.nvalid) continue;
        R out_phi[VEC], out_pi[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const R c = Pc.v[t][j];
            R nm[D], np[D];
            neighbours<D, VEC, TY>(Pm, Pc, Pn, left, right, S.nvalid, t, j, nm, np);
            if constexpr (UPDATE) {
                R ns;
                if constexpr (D == 3)
                    ns = nsum3(nm[0], np[0], nm[1], np[1], nm[2], np[2]);
                else
                    ns = nsum2(nm[0], np[0], nm[1], np[1]);
                kick_drift<D, UNIT>(c, ns, pic[t][j], A.k, out_pi[j], out_phi[j]);
            }
            if constexpr (DIAG) {
                if (S.active) site_diag<D>(c, pic[t][j], nm, np, A.dc, acc);
            }
        }
        if constexpr (UPDATE) {
            if (S.active) {
                store_vec<VEC>(phi_out + S.off[t], out_phi);
                store_vec<VEC>(pi_out + S.off[t], out_pi);
            }
        }
    }
}

// One wave's tile of one step (see the file header).  `tile` must be below
// A.ntiles and uniform across the wave.  The march is unrolled by four over a
// ring of four plane buffers, so no plane is ever copied between registers.
template <int D, int VEC, int TY, bool UPDATE, bool DIAG, bool UNIT = false, typename R = float>
__device__ __forceinline__ void step_tile(const StepArgsT<R>& A, int64_t tile)
{
    static_assert(D == 3 || TY == 1, "2D tiles have one row");
    const int lane = threadIdx.x & (kWave - 1);
    const TileSetup<TY> S = tile_setup<VEC, TY>(A.nx, A.Q, A.M, A.tiles_x, A.tiles_q, A.rows, tile);

    Plane<VEC, TY, R> P0, P1, P2, P3;
    R pi0[TY][VEC], pi1[TY][VEC];
    zero_plane(P0);
    zero_plane(P1);
    zero_plane(P2);
    zero_plane(P3);
    zero_rows<VEC, TY>(pi0);
    zero_rows<VEC, TY>(pi1);
    load_plane_values<VEC, TY>(A.phi_in, S.s0 - 1, S, P0);
    load_plane<D, VEC, TY>(A.phi_in, S.s0, S, P1);
    load_plane<D, VEC, TY>(A.phi_in, S.s0 + 1, S, P2);
    load_point<VEC, TY>(A.pi, S.s0, S, pi0);

    DiagAcc acc;
    acc.links[0] = acc.links[1] = acc.links[2] = 0u;
    acc.walls = acc.nonfinite = 0u;
    acc.area = acc.ek = 0.0;

    for (int64_t s = S.s0; s < S.s1; s += 4) {
        step_plane<D, VEC, TY, UPDATE, DIAG, UNIT>(A, S, s, P0, P1, P2, P3, pi0, pi1, acc);
        if (s + 1 >= S.s1) break;
        step_plane<D, VEC, TY, UPDATE, DIAG, UNIT>(A, S, s + 1, P1, P2, P3, P0, pi1, pi0, acc);
        if (s + 2 >= S.s1) break;
        step_plane<D, VEC, TY, UPDATE, DIAG, UNIT>(A, S, s + 2, P2, P3, P0, P1, pi0, pi1, acc);
        if (s + 3 >= S.s1) break;
        step_plane<D, VEC, TY, UPDATE, DIAG, UNIT>(A, S, s + 3, P3, P0, P1, P2, pi1, pi0, acc);
    }

    if constexpr (DIAG) {
        WavePartial w;
        w.links[0] = wave_sum_u32(acc.links[0]);
        w.links[1] = wave_sum_u32(acc.links[1]);
        w.links[2] = wave_sum_u32(acc.links[2]);
        w.walls = wave_sum_u32(acc.walls);
        w.nonfinite = wave_sum_u32(acc.nonfinite);
        w.pad = 0u;
        w.area = wave_sum_f64(acc.area);
        w.ek = wave_sum_f64(acc.ek);
        if (lane == 0) A.partials[tile] = w;
    }
}

template <int D, int VEC, int TY, bool UPDATE, bool DIAG, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_step(StepArgsT<R> A)
{
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block();
    if (tile >= A.ntiles) return;   // whole wave leaves; shuffles stay uniform
    step_tile<D, VEC, TY, UPDATE, DIAG, UNIT>(A, tile);
}

// SplitMix64 (Steele, Lea & Flood 2014) evaluated at counter i+1, top 24
// bits k mapped to (2k+1)/2^24 - 1.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fill_uniform(R* __restrict__ phi, int64_t count, uint64_t seed)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        const int32_t k = (int32_t)(z >> 40);
        phi[i] = (R)((float)(2 * k + 1 - (1 << 24)) * 0x1p-24f);   // exact in float
    }
}


// ---------------------------------------------------------------- adjoint --
//
// Reverse sweep of one step n of Eqs. (3)-(6).  The carried adjoint state is
// (mu, w): mu = dL/dphi^{n+1} and w = nu + deta*mu, the total adjoint of
// phi_dot^{n+1/2} (nu being its adjoint through later kicks).  Differentiating
// the kick and drift gives, per site,
//     mu^n    = mu^{n+1} + b_n (Lap w - V''(phi^n) w)     (Lap is symmetric)
//     w_{n-1} = a_n w + cw * mu^n                          (cw = deta; 0 on the
//                                                           last reverse step,
//                                                           which leaves nu = a w)
//     dL/dV0 += -b_n sum_i w_i d V'(phi_i)/dV0,  dV'/dV0 = 4 kc phi (kc phi^2 - 1)
// Same march and tiling as the forward kernel: w is the stencil field (read
// with halo, written to the other buffer), mu is updated in place and phi^n
// is read once.  20 bytes of HBM traffic per site.

template <typename R>
struct AdjArgsT {
    const R* w_in;
    R* w_out;
    R* mu;
    const R* phi_n;
    double* gacc;       // one accumulator per wave tile, persistent across steps
    int64_t nx, Q, M;
    int64_t tiles_x, tiles_q, ntiles;
    int64_t rows;
    R a, b, cw, F, kc, inv_dx2;
    double gscale;      // -4 kc b_n
};

// Plane s of a reverse tile (same ring scheme as step_plane).
template <int D, int VEC, int TY, bool UNIT, typename R>
__device__ __forceinline__ void adj_plane(const AdjArgsT<R>& A, const TileSetup<TY>& S, int64_t s,
                                          const Plane<VEC, TY, R>& Pm, const Plane<VEC, TY, R>& Pc,
                                          const Plane<VEC, TY, R>& Pn, Plane<VEC, TY, R>& Pnn,
                                          const R (&muc)[TY][VEC], R (&mun)[TY][VEC],
                                          const R (&phc)[TY][VEC], R (&phn)[TY][VEC],
                                          double& gsum)
{
    if (s + 1 < S.s1) {
        load_plane<D, VEC, TY>(A.w_in, s + 2, S, Pnn);
        load_point<VEC, TY>(A.mu, s + 1, S, mun);
        load_point<VEC, TY>(A.phi_n, s + 1, S, phn);
    }
    R left[TY], right[TY];
    x_neighbours<VEC, TY>(Pc, S, left, right);
    R* w_out = A.w_out + s * S.pstride;
    R* mu_out = A.mu + s * S.pstride;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        if (t >= S.nvalid) continue;
        R out_w[VEC], out_mu[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const R w = Pc.v[t][j];
            R nm[D], np[D];
            neighbours<D, VEC, TY>(Pm, Pc, Pn, left, right, S.nvalid, t, j, nm, np);
            R ns;
            if constexpr (D == 3)
                ns = nsum3(nm[0], np[0], nm[1], np[1], nm[2], np[2]);
            else
                ns = nsum2(nm[0], np[0], nm[1], np[1]);
            const R gp = adj_site<D, UNIT>(w, ns, muc[t][j], phc[t][j], A.a, A.b, A.cw, A.F, A.kc, A.inv_dx2,
                                           out_w[j], out_mu[j]);
            if (S.active) gsum += (double)gp;
        }
        if (S.active) {
            store_vec<VEC>(w_out + S.off[t], out_w);
            store_vec<VEC>(mu_out + S.off[t], out_mu);
        }
    }
}

template <int D, int VEC, int TY, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjArgsT<R> A)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block();
    if (tile >= A.ntiles) return;
    const TileSetup<TY> S = tile_setup<VEC, TY>(A.nx, A.Q, A.M, A.tiles_x, A.tiles_q, A.rows, tile);

    Plane<VEC, TY, R> P0, P1, P2, P3;
    R mu0[TY][VEC], mu1[TY][VEC], ph0[TY][VEC], ph1[TY][VEC];
    zero_plane(P0);
    zero_plane(P1);
    zero_plane(P2);
    zero_plane(P3);
    zero_rows<VEC, TY>(mu0);
    zero_rows<VEC, TY>(mu1);
    zero_rows<VEC, TY>(ph0);
    zero_rows<VEC, TY>(ph1);
    load_plane_values<VEC, TY>(A.w_in, S.s0 - 1, S, P0);
    load_plane<D, VEC, TY>(A.w_in, S.s0, S, P1);
    load_plane<D, VEC, TY>(A.w_in, S.s0 + 1, S, P2);
    load_point<VEC, TY>(A.mu, S.s0, S, mu0);
    load_point<VEC, TY>(A.phi_n, S.s0, S, ph0);

    double gsum = 0.0;
    for (int64_t s = S.s0; s < S.s1; s += 4) {
        adj_plane<D, VEC, TY, UNIT>(A, S, s, P0, P1, P2, P3, mu0, mu1, ph0, ph1, gsum);
        if (s + 1 >= S.s1) break;
        adj_plane<D, VEC, TY, UNIT>(A, S, s + 1, P1, P2, P3, P0, mu1, mu0, ph1, ph0, gsum);
        if (s + 2 >= S.s1) break;
        adj_plane<D, VEC, TY, UNIT>(A, S, s + 2, P2, P3, P0, P1, mu0, mu1, ph0, ph1, gsum);
        if (s + 3 >= S.s1) break;
        adj_plane<D, VEC, TY, UNIT>(A, S, s + 3, P3, P0, P1, P2, mu1, mu0, ph1, ph0, gsum);
    }
    gsum = wave_sum_f64(gsum);
    if (lane == 0) A.gacc[tile] += A.gscale * gsum;
}

// Seed of the reverse sweep and the loss sum V/V0 = (kc phi^2 - 1)^2 over the
// final field: mu = dL/dphi = 4 kc phi (kc phi^2 - 1), w = deta * mu (the
// final phi_dot does not enter the loss).  Fixed grid; one FP64 partial per
// workgroup.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_seed(const R* __restrict__ phi, int64_t count, R kc, R deta,
                                                      R* __restrict__ mu, R* __restrict__ w,
                                                      double* __restrict__ partial)
{
    __shared__ double sh[kBlock];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const R f = phi[i];
        const R q = f * f * kc - R(1);
        const R m = (R(4) * kc) * f * q;
        mu[i] = m;
        w[i] = deta * m;
        const double qd = (double)f * (double)f * (double)kc - 1.0;
        acc += qd * qd;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// ----------------------------------------- T steps per HBM pass (2D) --------
//
// Temporal blocking: T = 2, 3, 4 (and, in float32, 6 or 8) leapfrog steps
// per pass over HBM, with overlapped wave tiles.  A wave's 64 lanes hold 64*VEC consecutive sites; the first and
// last H = ceil(T/VEC) lanes are halo lanes whose sites belong to the
// neighbouring tiles.  Level k (step n+k-1) is computed for every lane from
// level k-1 of the lanes on either side (plain shuffles), so the sites within
// k of the wave's ends become stale at level k; halo lanes are never stored
// and H*VEC >= T keeps every owned site exact.  Along y the levels are
// pipelined inside the march: at iteration y level k computes row y-k+1 from
// level k-1 rows y-k .. y-k+2, so level k needs T-k extra rows on each side
// of the tile.  Only level T is written.  All levels use the single-step
// arithmetic, so the result is bitwise that of T single steps.

template <int T, typename R = float>
struct TBArgs {
    const R* phi_in;
    R* phi_out;
    const R* pi_in;
    R* pi_out;
    R* phi_lv[T];               // with ALL: phi^{n+k} of levels k = 1 .. T-1 (level T is phi_out);
                                // with MID: phi_lv[0] receives phi^{n+MID}
    R* pi_mid;                  // with MID: phi_dot^{n+MID-1/2}
    WavePartial* partials;
    int64_t nx, ny;
    int64_t tiles_x, ntiles;
    int64_t rows;
    int32_t yhalo = 0;          // 0: periodic in y; T: a y-slab stored with T halo rows below and above
    StepCoefT<R> k[T];
    DiagCoef dc;
};

__host__ __device__ __forceinline__ int64_t tb_owned_width_d(int vec, int T)
{
    const int H = (T + vec - 1) / vec;
    return (int64_t)(kWave - 2 * H) * vec;
}

template <int VEC, int T, typename R>
struct TBState {
    R in[4][VEC];              // phi^n rows, ring over the march
    R pin[2][VEC];             // phi_dot^{n-1/2} rows
    R lv[T][4][VEC];           // level k rows (k = 1 .. T-1 used)
    R pl[T][2][VEC];           // level k phi_dot rows
};

// Per-wave constants of a tile.  Row numbers are wave-uniform 32-bit values
// (a plane holds fewer than 2^31 sites), so all row arithmetic stays on the
// scalar unit.  Rows are read and written through raw buffer descriptors made
// per row (base = row start, size = row bytes): a lane's access is the
// descriptor plus its column offset, an access with size 0 or an offset past
// the row is dropped by the hardware, so every load and store is issued
// unconditionally and the memory counters the compiler waits on follow one
// straight-line pattern per iteration.
struct TBLane {
    uint32_t voff;             // byte offset of this lane's first site, wrapped into the row
    uint32_t soff;             // voff for owned lanes inside the lattice, else past the row
    int32_t s0, s1;            // output rows [s0, s1) of the tile
    uint32_t nx;
    uint32_t row_bytes;
    int32_t ny;
    int32_t dir;               // march direction of k_tb2d: +1 up (rising y), -1 down
    int32_t wrap_at, wrap_to;  // row after the last one in that direction, and its periodic image
    int32_t yoff;              // k_tb2d: stored row of row y is y + yoff (slab halo depth, else 0)
};

// Next rows to fetch, already wrapped into the stored rows ([0, ny), or
// [0, ny + 2T) for a slab with T halo rows per face); advanced by one row per
// iteration without division.
struct TBRows {
    int32_t phi, pi;
};

__device__ __forceinline__ int32_t next_row(int32_t r, int32_t ny)
{
    return r + 1 == ny ? 0 : r + 1;
}

// Next row of a k_tb2d march in its direction, periodic.
__device__ __forceinline__ int32_t step_row(int32_t r, const TBLane& L)
{
    const int32_t n = r + L.dir;
    return n == L.wrap_at ? L.wrap_to : n;
}

// Any row number into [0, ny) (tile set-up only).
__device__ __forceinline__ int32_t wrap_row(int32_t r, int32_t ny)
{
    r %= ny;
    return r < 0 ? r + ny : r;
}

// Word 3 of a raw (unswizzled, stride 0) buffer descriptor on CDNA.
constexpr int kRawBufferWord3 = 0x00020000;

// Offset that no row reaches (rows are shorter than 2^30 bytes).
constexpr uint32_t kPastRow = 0xFFFFFFF0u;

// Raw buffer descriptor over [base, base + bytes): lane accesses at byte
// offsets at or past `bytes` are dropped (loads return 0).
template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const R* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(base), (short)0, (int)bytes, kRawBufferWord3);
}

__device__ __forceinline__ double u64_as_double(uint32_t lo, uint32_t hi)
{
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// VEC values of this lane at byte offset voff of the span [base, base+bytes).
template <int VEC, typename R>
__device__ __forceinline__ void buf_load(const R* base, uint32_t bytes, uint32_t voff, R (&v)[VEC])
{
    static_assert(VEC * sizeof(R) <= 16, "at most 16 bytes per lane and access");
    const __amdgpu_buffer_rsrc_t r = span_rsrc(base, bytes);
    if constexpr (sizeof(R) == 8 && VEC == 2) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
        v[0] = u64_as_double(t[0], t[1]);
        v[1] = u64_as_double(t[2], t[3]);
    } else if constexpr (sizeof(R) == 8) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
        v[0] = u64_as_double(t[0], t[1]);
    } else if constexpr (VEC == 4) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = __uint_as_float(t[j]);
    } else if constexpr (VEC == 2) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
        v[0] = __uint_as_float(t[0]);
        v[1] = __uint_as_float(t[1]);
    } else {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
    }
}

// Cache policy of the multi-step passes' field stores (0: the default
// write-back policy; a translation unit may define another before including
// this header).
#ifndef PRS_STORE_AUX
#define PRS_STORE_AUX 0
#endif

template <int VEC, typename R>
__device__ __forceinline__ void buf_store(R* base, uint32_t bytes, uint32_t soff, const R (&v)[VEC])
{
    static_assert(VEC * sizeof(R) <= 16, "at most 16 bytes per lane and access");
    const __amdgpu_buffer_rsrc_t r = span_rsrc(base, bytes);
    constexpr int W = VEC * (int)sizeof(R) / 4;   // 32-bit words per lane
    __attribute__((ext_vector_type(W == 1 ? 2 : W))) unsigned int t;
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        if constexpr (sizeof(R) == 8) {
            const uint64_t b = __builtin_bit_cast(uint64_t, v[j]);
            t[2 * j] = (uint32_t)b;
            t[2 * j + 1] = (uint32_t)(b >> 32);
        } else {
            t[j] = __float_as_uint(v[j]);
        }
    }
    if constexpr (W == 4) {
        __builtin_amdgcn_raw_buffer_store_b128(t, r, soff, 0, PRS_STORE_AUX);
    } else if constexpr (W == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(t, r, soff, 0, PRS_STORE_AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(t[0], r, soff, 0, PRS_STORE_AUX);
    }
}

// Row `row` of a 2D field through a descriptor spanning that row.
template <int VEC, typename R>
__device__ __forceinline__ void tb_load(const R* f, int32_t row, const TBLane& L, uint32_t bytes, R (&v)[VEC])
{
    buf_load<VEC>(f + (size_t)(uint32_t)row * L.nx, bytes, L.voff, v);
}

template <int VEC, typename R>
__device__ __forceinline__ void tb_store(R* f, int32_t row, const TBLane& L, uint32_t bytes, const R (&v)[VEC])
{
    buf_store<VEC>(f + (size_t)(uint32_t)row * L.nx, bytes, L.soff, v);
}

// Iteration i of the march (upward: y = s0 - T + 1 + i; level k computes
// row s0 - T - k + 2 + i; a downward march mirrors the rows in the tile).
// Level k has work from i = 2(k-1) on, the last
// iteration is i = last for every level.  CHECK skips the levels that have no
// row yet (the first 2T-2 iterations); without it those levels run on rows
// that only ever feed rows outside the tile, which are never stored.
template <int VEC, int T, bool DIAG, bool UNIT, bool CHECK, int U, bool ALL, typename R, int MID = 0>
__device__ __forceinline__ void tb_iter(const TBArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                        TBRows& rw, TBState<VEC, T, R>& S, DiagAcc& acc)
{
    // prefetch phi^n row y+2 and phi_dot row y+1 for the next iteration
    // (none after the last: size 0)
    const uint32_t nb = i < last ? L.row_bytes : 0u;
    tb_load<VEC>(A.phi_in, rw.phi, L, nb, S.in[(U + 2) & 3]);
    tb_load<VEC>(A.pi_in, rw.pi, L, nb, S.pin[(U + 1) & 1]);
    rw.phi = step_row(rw.phi, L);
    rw.pi = step_row(rw.pi, L);
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * (k - 1)) continue;
        const R* cm;
        const R* cc;
        const R* cp;
        const R* pp;
        if (k == 1) {
            cm = S.in[(U + 3) & 3];
            cc = S.in[U & 3];
            cp = S.in[(U + 1) & 3];
            pp = S.pin[U & 1];
        } else {
            cm = S.lv[k - 1][(U + 2) & 3];
            cc = S.lv[k - 1][(U + 3) & 3];
            cp = S.lv[k - 1][U & 3];
            pp = S.pl[k - 1][(U + 1) & 1];
        }
        R left = from_left_lane(cc[VEC - 1]);
        R right = from_right_lane(cc[0]);
        R out_phi[VEC], out_pi[VEC];
        // level 1 row y is inside the tile for i in [T-1, T-1 + s1 - s0)
        const bool diag_row = DIAG && k == 1 && i >= T - 1 && i < T - 1 + (L.s1 - L.s0);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const R c = cc[j];
            const R xm = j > 0 ? cc[j > 0 ? j - 1 : 0] : left;
            const R xp = j < VEC - 1 ? cc[j < VEC - 1 ? j + 1 : j] : right;
            kick_drift<2, UNIT>(c, nsum2(xm, xp, cm[j], cp[j]), pp[j], A.k[k - 1], out_pi[j], out_phi[j]);
            if constexpr (DIAG) {
                if (diag_row && L.soff != kPastRow) {
                    const R nm[2] = {xm, cm[j]};
                    const R np[2] = {xp, cp[j]};
                    site_diag<2>(c, pp[j], nm, np, A.dc, acc);
                }
            }
        }
        if (k < T) {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.lv[k < T ? k : 0][U & 3][j] = out_phi[j];
                S.pl[k < T ? k : 0][U & 1][j] = out_pi[j];
            }
            if constexpr (ALL) {
                // level k: march row e = i - (T + k - 2) of the tile, stored when inside [0, s1 - s0)
                const int32_t e = i - (T + k - 2);
                const bool in = e >= 0 && e < L.s1 - L.s0;
                const int32_t row = (L.dir > 0 ? L.s0 + e : L.s1 - 1 - e) + L.yoff;
                tb_store<VEC>(A.phi_lv[k < T ? k - 1 : 0], in ? row : L.s0, L, in ? L.row_bytes : 0u, out_phi);
            }
            if constexpr (MID > 0) {
                if (k == MID) {
                    // the state after MID steps, (phi, phi_dot) of the same row
                    const int32_t e = i - (T + k - 2);
                    const bool in = e >= 0 && e < L.s1 - L.s0;
                    const int32_t row = (L.dir > 0 ? L.s0 + e : L.s1 - 1 - e) + L.yoff;
                    tb_store<VEC>(A.phi_lv[0], in ? row : L.s0, L, in ? L.row_bytes : 0u, out_phi);
                    tb_store<VEC>(A.pi_mid, in ? row : L.s0, L, in ? L.row_bytes : 0u, out_pi);
                }
            }
        } else {
            // level T: march row e = i - (2T - 2) of the tile, inside it once i >= 2T - 2
            const int32_t e = i - (2 * T - 2);
            const int32_t row = (L.dir > 0 ? L.s0 + e : L.s1 - 1 - e) + L.yoff;
            const uint32_t sb = (!CHECK || i >= 2 * T - 2) ? L.row_bytes : 0u;
            tb_store<VEC>(A.phi_out, CHECK && i < 2 * T - 2 ? L.s0 : row, L, sb, out_phi);
            tb_store<VEC>(A.pi_out, CHECK && i < 2 * T - 2 ? L.s0 : row, L, sb, out_pi);
        }
    }
}

// Iterations i .. i+3 (i a multiple of 4, so ring slots are compile-time);
// false once the last iteration has run.
template <int VEC, int T, bool DIAG, bool UNIT, bool CHECK, bool ALL, typename R, int MID = 0>
__device__ __forceinline__ bool tb_group(const TBArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                         TBRows& rw, TBState<VEC, T, R>& S, DiagAcc& acc)
{
    tb_iter<VEC, T, DIAG, UNIT, CHECK, 0, ALL, R, MID>(A, L, i, last, rw, S, acc);
    if (i + 1 > last) return false;
    tb_iter<VEC, T, DIAG, UNIT, CHECK, 1, ALL, R, MID>(A, L, i + 1, last, rw, S, acc);
    if (i + 2 > last) return false;
    tb_iter<VEC, T, DIAG, UNIT, CHECK, 2, ALL, R, MID>(A, L, i + 2, last, rw, S, acc);
    if (i + 3 > last) return false;
    tb_iter<VEC, T, DIAG, UNIT, CHECK, 3, ALL, R, MID>(A, L, i + 3, last, rw, S, acc);
    return i + 4 <= last;
}

// One wave's tile of a T-step pass; `tile` must be below A.ntiles and
// wave-uniform.  ALL also stores the fields of the intermediate steps
// (phi_lv), as the recomputation of the adjoint needs them.
template <int VEC, int T, bool DIAG, bool UNIT = false, bool ALL = false, typename R = float, int MID = 0>
__device__ __forceinline__ void tb_tile(const TBArgs<T, R>& A, int64_t tile)
{
    constexpr int H = (T + VEC - 1) / VEC;        // halo lanes per side
    constexpr int W = (kWave - 2 * H) * VEC;       // owned sites per wave
    constexpr int WARM = (2 * T - 2 + 3) / 4;      // groups that hold pipeline fill
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t ts = tl / (uint32_t)A.tiles_x;
    TBLane L;
    L.nx = (uint32_t)A.nx;
    L.ny = (int32_t)A.ny;
    L.row_bytes = L.nx * (uint32_t)sizeof(R);
    const int32_t rows = (int32_t)A.rows;
    // x0 < nx + 64 VEC fits in 32 bits; lanes past a narrow lattice wrap
    // more than once and only load
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    L.voff = (uint32_t)wrap_row(x0, (int32_t)L.nx) * (uint32_t)sizeof(R);
    L.soff = (lane >= H && lane < kWave - H && x0 < (int32_t)L.nx) ? L.voff : kPastRow;
    L.s0 = (int32_t)ts * rows;
    L.s1 = L.s0 + rows < L.ny ? L.s0 + rows : L.ny;
    // Odd row tiles march down, so that two neighbouring tiles start at
    // their common edge together or end there together: the 2T - 2 halo
    // rows each reads of the other's rows are then fetched from HBM about
    // once and found in L2 by the second reader.  The y-neighbour sum is
    // symmetric, so the results are the same bits either way.  Diagnostic
    // passes march up (their links point to rising y).
    L.dir = (DIAG || (ts & 1u) == 0u) ? 1 : -1;
    // A slab reads its T halo rows instead of wrapping around: its rows are
    // stored T up, and the march never leaves them except by loads of size 0
    // (the wrap below keeps even those inside the buffer).
    L.yoff = A.yhalo;
    const int32_t stored = L.ny + 2 * A.yhalo;
    L.wrap_at = L.dir > 0 ? stored : -1;
    L.wrap_to = L.dir > 0 ? 0 : stored - 1;
    auto yrow = [&](int32_t y) { return A.yhalo ? y + A.yhalo : wrap_row(y, L.ny); };

    TBState<VEC, T, R> S;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            S.in[a][j] = R(0);
#pragma unroll
            for (int k = 0; k < T; ++k) S.lv[k][a][j] = R(0);
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            S.pin[a][j] = R(0);
#pragma unroll
            for (int k = 0; k < T; ++k) S.pl[k][a][j] = R(0);
        }

    // iteration 0 (y0 = T - 1 rows before the tile's first row in the march
    // direction) needs phi^n rows y0 - dir .. y0 + dir and phi_dot row y0
    const int32_t d = L.dir;
    const int32_t y0 = d > 0 ? L.s0 - T + 1 : L.s1 + T - 2;
    tb_load<VEC>(A.phi_in, yrow(y0 - d), L, L.row_bytes, S.in[3]);
    tb_load<VEC>(A.phi_in, yrow(y0), L, L.row_bytes, S.in[0]);
    tb_load<VEC>(A.phi_in, yrow(y0 + d), L, L.row_bytes, S.in[1]);
    tb_load<VEC>(A.pi_in, yrow(y0), L, L.row_bytes, S.pin[0]);
    TBRows rw;
    rw.phi = yrow(y0 + 2 * d);
    rw.pi = yrow(y0 + d);

    DiagAcc acc;
    acc.links[0] = acc.links[1] = acc.links[2] = 0u;
    acc.walls = acc.nonfinite = 0u;
    acc.area = acc.ek = 0.0;

    const int32_t last = (L.s1 - L.s0) + 2 * T - 3;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tb_group<VEC, T, DIAG, UNIT, true, ALL, R, MID>(A, L, i, last, rw, S, acc);
        i += 4;
    }
    while (more) {
        more = tb_group<VEC, T, DIAG, UNIT, false, ALL, R, MID>(A, L, i, last, rw, S, acc);
        i += 4;
    }

    if constexpr (DIAG) {
        WavePartial w;
        w.links[0] = wave_sum_u32(acc.links[0]);
        w.links[1] = wave_sum_u32(acc.links[1]);
        w.links[2] = 0u;
        w.walls = wave_sum_u32(acc.walls);
        w.nonfinite = wave_sum_u32(acc.nonfinite);
        w.pad = 0u;
        w.area = wave_sum_f64(acc.area);
        w.ek = wave_sum_f64(acc.ek);
        if (lane == 0) A.partials[tile] = w;
    }
}

// Waves per SIMD the register allocation of k_tb2d must leave room for: the
// float32 eight-step pass with two sites per lane fits 128 VGPRs (four waves)
// without spilling and is held there.
constexpr int tb2d_min_waves(int vec, int T, int esize)
{
    return (esize == 4 && vec == 2 && T == 8) ? 4 : 1;
}

template <int VEC, int T, bool DIAG, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(tb2d_min_waves(VEC, T, (int)sizeof(R))))) void k_tb2d(TBArgs<T, R> A)
{
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    tb_tile<VEC, T, DIAG, UNIT>(A, tile);
}

// The T-step pass also storing the state after T/2 steps (the pass starts
// of the fused adjoint's reverse passes, two per forward pass).
template <int VEC, int T, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(tb2d_min_waves(VEC, T, (int)sizeof(R))))) void k_tb2d_mid(TBArgs<T, R> A)
{
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    tb_tile<VEC, T, false, UNIT, false, R, T / 2>(A, tile);
}

// The T-step pass storing every step's field (adjoint recomputation).
template <int VEC, int T, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tb2d_all(TBArgs<T, R> A)
{
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    tb_tile<VEC, T, false, UNIT, true>(A, tile);
}

// ------------------------------- reverse sweep, T steps per pass (2D) ------
//
// T reverse steps m, m-1, ..., m-T+1 of the adjoint (Eqs. 3-6 differentiated,
// as in k_adjoint) in one pass, with the overlapped tiles and the pipelined
// y-march of the forward passes: level k is reverse step m-k+1, w is the
// stencil field and mu the pointwise one, and level k also reads phi^{m-k+1}
// (its own field).  w and mu are read from w_in, mu_in and written after the
// last level to w_out, mu_out, which must be other buffers (neighbouring
// tiles read the rows this tile overlaps).  Each level's dL/dV0 sum is kept
// apart and added with its own coefficient.  Per site every level evaluates
// exactly the arithmetic of k_adjoint, so w and mu are bitwise those of
// single reverse steps; dL/dV0 differs in summation order only.

template <int T, typename R = float>
struct TBAArgs {
    const R* w_in;
    R* w_out;
    const R* mu_in;
    R* mu_out;
    const R* phi[T];            // phi^{m-k+1} for level k = 1 .. T
    double* gacc;               // one accumulator per wave tile of this pass shape
    int64_t nx, ny;
    int64_t tiles_x, ntiles;
    int64_t rows;
    R a[T], b[T], cw[T], F[T];  // F carries the step's a(eta)^beta
    R kc, inv_dx2;
    double gscale[T];
};

template <int VEC, int T, typename R>
struct TBAState {
    R in[4][VEC];               // w rows, ring over the march
    R mi[2][VEC];               // mu rows
    R lv[T][4][VEC];            // level k w rows (k = 1 .. T-1)
    R ml[T][2][VEC];            // level k mu rows
    R ph[T][2][VEC];            // phi row of each level, one iteration ahead
};

template <int VEC, int T, bool UNIT, bool CHECK, int U, typename R>
__device__ __forceinline__ void tba_iter(const TBAArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                         TBRows& rw, int32_t (&prow)[T], TBAState<VEC, T, R>& S,
                                         double (&gs)[T])
{
    // prefetch for the next iteration: w row y+2, mu row y+1 and, for every
    // level k, the phi row it computes next
    const uint32_t nb = i < last ? L.row_bytes : 0u;
    tb_load<VEC>(A.w_in, rw.phi, L, nb, S.in[(U + 2) & 3]);
    tb_load<VEC>(A.mu_in, rw.pi, L, nb, S.mi[(U + 1) & 1]);
    rw.phi = step_row(rw.phi, L);
    rw.pi = step_row(rw.pi, L);
#pragma unroll
    for (int k = 0; k < T; ++k) {
        tb_load<VEC>(A.phi[k], prow[k], L, nb, S.ph[k][(U + 1) & 1]);
        prow[k] = step_row(prow[k], L);
    }
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * (k - 1)) continue;
        const R* cm;
        const R* cc;
        const R* cp;
        const R* mp;
        if (k == 1) {
            cm = S.in[(U + 3) & 3];
            cc = S.in[U & 3];
            cp = S.in[(U + 1) & 3];
            mp = S.mi[U & 1];
        } else {
            cm = S.lv[k - 1][(U + 2) & 3];
            cc = S.lv[k - 1][(U + 3) & 3];
            cp = S.lv[k - 1][U & 3];
            mp = S.ml[k - 1][(U + 1) & 1];
        }
        const R* ph = S.ph[k - 1][U & 1];
        // level k row s0 + i - (T + k - 2) counts for dL/dV0 when inside [s0, s1)
        const int32_t e = i - (T + k - 2);
        const bool own_row = e >= 0 && e < L.s1 - L.s0;
        const R left = from_left_lane(cc[VEC - 1]);
        const R right = from_right_lane(cc[0]);
        R out_w[VEC], out_mu[VEC];
        double g = 0.0;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const R w = cc[j];
            const R xm = j > 0 ? cc[j > 0 ? j - 1 : 0] : left;
            const R xp = j < VEC - 1 ? cc[j < VEC - 1 ? j + 1 : j] : right;
            const R gp = adj_site<2, UNIT>(w, nsum2(xm, xp, cm[j], cp[j]), mp[j], ph[j], A.a[k - 1], A.b[k - 1],
                                           A.cw[k - 1], A.F[k - 1], A.kc, A.inv_dx2, out_w[j], out_mu[j]);
            g += (double)gp;
        }
        // own_row is wave-uniform; lanes outside the owned columns add g * 0
        if (own_row) gs[k - 1] = fma(g, L.soff != kPastRow ? 1.0 : 0.0, gs[k - 1]);
        if (k < T) {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.lv[k < T ? k : 0][U & 3][j] = out_w[j];
                S.ml[k < T ? k : 0][U & 1][j] = out_mu[j];
            }
        } else {
            const int32_t e = i - (2 * T - 2);
            const int32_t row = L.dir > 0 ? L.s0 + e : L.s1 - 1 - e;
            const uint32_t sb = (!CHECK || i >= 2 * T - 2) ? L.row_bytes : 0u;
            tb_store<VEC>(A.w_out, CHECK && i < 2 * T - 2 ? L.s0 : row, L, sb, out_w);
            tb_store<VEC>(A.mu_out, CHECK && i < 2 * T - 2 ? L.s0 : row, L, sb, out_mu);
        }
    }
}

template <int VEC, int T, bool UNIT, bool CHECK, typename R>
__device__ __forceinline__ bool tba_group(const TBAArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                          TBRows& rw, int32_t (&prow)[T], TBAState<VEC, T, R>& S,
                                          double (&gs)[T])
{
    tba_iter<VEC, T, UNIT, CHECK, 0>(A, L, i, last, rw, prow, S, gs);
    if (i + 1 > last) return false;
    tba_iter<VEC, T, UNIT, CHECK, 1>(A, L, i + 1, last, rw, prow, S, gs);
    if (i + 2 > last) return false;
    tba_iter<VEC, T, UNIT, CHECK, 2>(A, L, i + 2, last, rw, prow, S, gs);
    if (i + 3 > last) return false;
    tba_iter<VEC, T, UNIT, CHECK, 3>(A, L, i + 3, last, rw, prow, S, gs);
    return i + 4 <= last;
}

template <int VEC, int T, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tba2d(TBAArgs<T, R> A)
{
    constexpr int H = (T + VEC - 1) / VEC;
    constexpr int W = (kWave - 2 * H) * VEC;
    constexpr int WARM = (2 * T - 2 + 3) / 4;
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t ts = tl / (uint32_t)A.tiles_x;
    TBLane L;
    L.nx = (uint32_t)A.nx;
    L.ny = (int32_t)A.ny;
    L.row_bytes = L.nx * (uint32_t)sizeof(R);
    const int32_t rows = (int32_t)A.rows;
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    L.voff = (uint32_t)wrap_row(x0, (int32_t)L.nx) * (uint32_t)sizeof(R);
    L.soff = (lane >= H && lane < kWave - H && x0 < (int32_t)L.nx) ? L.voff : kPastRow;
    L.s0 = (int32_t)ts * rows;
    L.s1 = L.s0 + rows < L.ny ? L.s0 + rows : L.ny;
    // odd row tiles march down, as in k_tb2d (periodic: no halo rows)
    L.dir = (ts & 1u) == 0u ? 1 : -1;
    L.yoff = 0;
    L.wrap_at = L.dir > 0 ? L.ny : -1;
    L.wrap_to = L.dir > 0 ? 0 : L.ny - 1;

    TBAState<VEC, T, R> S;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            S.in[a][j] = R(0);
#pragma unroll
            for (int k = 0; k < T; ++k) S.lv[k][a][j] = R(0);
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            S.mi[a][j] = R(0);
#pragma unroll
            for (int k = 0; k < T; ++k) S.ml[k][a][j] = S.ph[k][a][j] = R(0);
        }

    // iteration 0 (y0 = T - 1 rows before the tile's first row in the march
    // direction d): w rows y0 - d .. y0 + d, mu row y0, and the phi row of
    // every level (level k computes row y0 - (k - 1) d)
    const int32_t d = L.dir;
    const int32_t y0 = d > 0 ? L.s0 - T + 1 : L.s1 + T - 2;
    tb_load<VEC>(A.w_in, wrap_row(y0 - d, L.ny), L, L.row_bytes, S.in[3]);
    tb_load<VEC>(A.w_in, wrap_row(y0, L.ny), L, L.row_bytes, S.in[0]);
    tb_load<VEC>(A.w_in, wrap_row(y0 + d, L.ny), L, L.row_bytes, S.in[1]);
    tb_load<VEC>(A.mu_in, wrap_row(y0, L.ny), L, L.row_bytes, S.mi[0]);
    int32_t prow[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        tb_load<VEC>(A.phi[k], wrap_row(y0 - k * d, L.ny), L, L.row_bytes, S.ph[k][0]);
        prow[k] = wrap_row(y0 - (k - 1) * d, L.ny);
    }
    TBRows rw;
    rw.phi = wrap_row(y0 + 2 * d, L.ny);
    rw.pi = wrap_row(y0 + d, L.ny);
    double gs[T];
#pragma unroll
    for (int k = 0; k < T; ++k) gs[k] = 0.0;

    const int32_t last = (L.s1 - L.s0) + 2 * T - 3;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tba_group<VEC, T, UNIT, true>(A, L, i, last, rw, prow, S, gs);
        i += 4;
    }
    while (more) {
        more = tba_group<VEC, T, UNIT, false>(A, L, i, last, rw, prow, S, gs);
        i += 4;
    }
    double gsum = 0.0;
#pragma unroll
    for (int k = 0; k < T; ++k) gsum += A.gscale[k] * wave_sum_f64(gs[k]);
    if (lane == 0) A.gacc[tile] += gsum;
}

// ---------------- reverse sweep recomputing its fields, T steps per pass (2D) --
//
// The reverse pass of k_tba2d without the stored fields: it reads the state
// (phi^s, phi_dot^{s-1/2}) the forward held at the pass's first step s and
// recomputes phi^{s+1} .. phi^{s+T-1} itself, as forward levels 1 .. T-1 of
// the forward passes' pipeline (kick_drift, the same arithmetic, so the same
// bits), while reverse levels 1 .. T run the steps s+T-1 .. s on them (the
// arithmetic of k_adjoint).  Nothing but the pass-start state and (w, mu)
// crosses memory: 24 B per site per pass in float32 instead of the 16 + 4T B
// of k_tba2d plus the 8 + 4T B of storing every step's field.
//
// Rows march up.  With y the newest level-0 row of iteration i (y = y0 + i),
// forward level j computes row y - j, reverse level 1 row y - T + 1 and
// reverse level k row y - T - k + 2 from reverse level k-1 and forward level
// T-k, whose row was computed 2k - 2 iterations earlier and waits in that
// level's register ring (2T - 2j - 1 rows deep for level j).  The final
// level writes row y - 2T + 2; a tile of n output rows runs n + 4T - 4
// iterations, starting with y0 = s0 - 2T + 2.  Lanes: the forward levels
// shrink the valid lanes by T - 1 sites per side and the reverse levels by T
// more, so a wave owns its middle 64 VEC - 2 (2T - 1) sites... rounded to
// whole lanes: H = ceil((2T - 1)/VEC) halo lanes per side.
//
// dL/dV0 is summed per level and lane in the field precision over one group
// of iterations and then added to a double per level; the gradient fields
// do not depend on it.

// Rows a ring holds: level 0 of phi keeps 2T rows (the oldest read 2T - 2
// iterations after it was loaded, one prefetched), forward level j
// max(3, 2T - 2j - 1) (its successor reads three rows, reverse level T-j the
// row of 2T - 2j - 2 iterations ago), the top level one.  Powers of two, so
// that the unrolled iterations address them with compile-time slots.
__host__ __device__ constexpr int tbf_pow2(int v) { return v <= 1 ? 1 : v <= 2 ? 2 : v <= 4 ? 4 : v <= 8 ? 8 : 16; }
__host__ __device__ constexpr int tbf_ring0(int T) { return tbf_pow2(2 * T); }
__host__ __device__ constexpr int tbf_ring(int T, int j)
{
    return j == T - 1 ? 1 : tbf_pow2(2 * T - 2 * j - 1 > 3 ? 2 * T - 2 * j - 1 : 3);
}
__host__ __device__ constexpr int tbf_halo(int vec, int T) { return (2 * T - 1 + vec - 1) / vec; }

template <int T, typename R = float>
struct TBFArgs {
    const R* phi_s;             // phi^s (the pass-start field)
    const R* pi_s;              // phi_dot^{s-1/2}
    const R* w_in;
    R* w_out;
    const R* mu_in;
    R* mu_out;
    double* gacc;               // one accumulator per wave tile
    int64_t nx, ny;
    int64_t tiles_x, ntiles;
    int64_t rows;
    StepCoefT<R> k[T];          // forward level j runs step s + j - 1 with k[j-1] (j = 1 .. T-1)
    R a[T], b[T], cw[T], F[T];  // reverse level k runs step s + T - k
    R kc, inv_dx2;
    double gscale[T];
};

template <int VEC, int T, typename R>
struct TBFState {
    R f0[tbf_ring0(T)][VEC];    // level 0 phi rows
    R p0[2][VEC];               // level 0 phi_dot rows
    R fl[T][8][VEC];            // forward level j phi rows (ring tbf_ring(T, j))
    R pl[T][2][VEC];            // forward level j phi_dot rows (j = 1 .. T-2)
    R wi[4][VEC];               // w_in rows
    R mi[2][VEC];               // mu_in rows
    R rw[T][4][VEC];            // reverse level k w rows (k = 1 .. T-1)
    R rm[T][2][VEC];            // reverse level k mu rows
};

struct TBFRows {
    int32_t phi, pi, w, mu;     // next rows to fetch, wrapped into [0, ny)
};

// One site of a reverse level: adj_site's update of (w, mu), with the
// dL/dV0 term's phi (kc phi^2 - 1) returned for the caller to accumulate.
template <bool UNIT, typename R>
__device__ __forceinline__ R adj_site_pq(R w, R s, R mu, R phi, R a, R b, R cw, R F, R kc, R inv_dx2, R& w_new,
                                         R& mu_new)
{
    const R pk = UNIT ? phi : phi * kc;
    const R q = fmar(pk, phi, R(-1));
    const R c1 = fmar(R(2), F, UNIT ? R(4) : R(4) * inv_dx2);
    const R t = fmar(R(3) * F, q, c1);
    const R x = fmar(-w, t, UNIT ? s : s * inv_dx2);
    mu_new = fmar(b, x, mu);
    w_new = fmar(cw, mu_new, a * w);
    return phi * q;
}

// The 2D neighbour sum of element j of a row whose x-neighbours across the
// lane boundary are `left` and `right`; the shifted value comes first in
// each pair so that the DPP shift folds into the add (same bits: each pair
// is one commutative addition).
template <int VEC, typename R>
__device__ __forceinline__ R row_nsum(const R* cc, R left, R right, int j, R ym, R yp)
{
    const R xm = j > 0 ? cc[j > 0 ? j - 1 : 0] : left;
    const R xp = j < VEC - 1 ? cc[j < VEC - 1 ? j + 1 : j] : right;
    const R xs = j == VEC - 1 ? (xp + xm) : (xm + xp);
    return xs + (ym + yp);
}

template <int VEC, int T, bool UNIT, bool CHECK, int U, typename R>
__device__ __forceinline__ void tbf_iter(const TBFArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                         int32_t n_out, TBFRows& rw, TBFState<VEC, T, R>& S, R (&g32)[T])
{
    constexpr int R0 = tbf_ring0(T);
    // prefetch for the next iteration: phi^s row y+1, phi_dot row y, w_in row
    // y-T+3, mu_in row y-T+2 (none after the last iteration: size 0)
    const uint32_t nb = i < last ? L.row_bytes : 0u;
    tb_load<VEC>(A.phi_s, rw.phi, L, nb, S.f0[(U + 1) & (R0 - 1)]);
    tb_load<VEC>(A.pi_s, rw.pi, L, nb, S.p0[U & 1]);
    tb_load<VEC>(A.w_in, rw.w, L, nb, S.wi[U & 3]);
    tb_load<VEC>(A.mu_in, rw.mu, L, nb, S.mi[U & 1]);
    rw.phi = next_row(rw.phi, L.ny);
    rw.pi = next_row(rw.pi, L.ny);
    rw.w = next_row(rw.w, L.ny);
    rw.mu = next_row(rw.mu, L.ny);

    // forward levels j = 1 .. T-1: row y - j
#pragma unroll
    for (int j = 1; j < T; ++j) {
        if (CHECK && i < 2 * j) continue;
        const R* cm;
        const R* cc;
        const R* cp;
        const R* pp;
        if (j == 1) {
            cm = S.f0[(U + R0 - 2) & (R0 - 1)];
            cc = S.f0[(U + R0 - 1) & (R0 - 1)];
            cp = S.f0[U & (R0 - 1)];
            pp = S.p0[(U + 1) & 1];
        } else {
            constexpr int RP = 8;
            const int rp = tbf_ring(T, j > 1 ? j - 1 : 1) - 1;
            cm = S.fl[j - 1][(U + RP - 2) & rp];
            cc = S.fl[j - 1][(U + RP - 1) & rp];
            cp = S.fl[j - 1][U & rp];
            pp = S.pl[j - 1][(U + 1) & 1];
        }
        const R left = from_left_lane(cc[VEC - 1]);
        const R right = from_right_lane(cc[0]);
        const int rj = tbf_ring(T, j) - 1;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            R pn, fn;
            kick_drift<2, UNIT>(cc[e], row_nsum<VEC>(cc, left, right, e, cm[e], cp[e]), pp[e], A.k[j - 1], pn, fn);
            S.fl[j][U & rj][e] = fn;
            if (j < T - 1) S.pl[j][U & 1][e] = pn;
        }
    }

    // reverse levels k = 1 .. T: row y - T - k + 2
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * T + 2 * k - 4) continue;
        const R* cm;
        const R* cc;
        const R* cp;
        const R* mp;
        if (k == 1) {
            cm = S.wi[(U + 1) & 3];
            cc = S.wi[(U + 2) & 3];
            cp = S.wi[(U + 3) & 3];
            mp = S.mi[(U + 1) & 1];
        } else {
            cm = S.rw[k - 1][(U + 2) & 3];
            cc = S.rw[k - 1][(U + 3) & 3];
            cp = S.rw[k - 1][U & 3];
            mp = S.rm[k - 1][(U + 1) & 1];
        }
        // forward level T-k's row of 2k - 2 iterations ago
        const R* ph;
        if (k == T) {
            ph = S.f0[(U + R0 - (2 * T - 2)) & (R0 - 1)];
        } else {
            constexpr int RP = 8;
            ph = S.fl[T - k][(U + RP - (2 * k - 2)) & (tbf_ring(T, T - k) - 1)];
        }
        const R left = from_left_lane(cc[VEC - 1]);
        const R right = from_right_lane(cc[0]);
        // row y - T - k + 2 is output row e of the tile when inside [0, n_out)
        const int32_t e_row = i - (3 * T + k - 4);
        const bool own_row = e_row >= 0 && e_row < n_out;
        R out_w[VEC], out_mu[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const R pq = adj_site_pq<UNIT>(cc[e], row_nsum<VEC>(cc, left, right, e, cm[e], cp[e]), mp[e], ph[e],
                                           A.a[k - 1], A.b[k - 1], A.cw[k - 1], A.F[k - 1], A.kc, A.inv_dx2,
                                           out_w[e], out_mu[e]);
            if (own_row) g32[k - 1] = fmar(cc[e], pq, g32[k - 1]);
        }
        if (k < T) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                S.rw[k < T ? k : 0][U & 3][e] = out_w[e];
                S.rm[k < T ? k : 0][U & 1][e] = out_mu[e];
            }
        } else {
            const int32_t er = i - (4 * T - 4);
            const uint32_t sb = (!CHECK || er >= 0) ? L.row_bytes : 0u;
            const int32_t row = L.s0 + (er >= 0 ? er : 0);
            tb_store<VEC>(A.w_out, row, L, sb, out_w);
            tb_store<VEC>(A.mu_out, row, L, sb, out_mu);
        }
    }
}

// Iterations i .. i+U-1 (U the level-0 ring length, so ring slots are
// compile-time); false once the last iteration has run.  The group's
// dL/dV0 partials are then added to the per-level doubles of owned lanes.
template <int VEC, int T, bool UNIT, bool CHECK, typename R, int... Us>
__device__ __forceinline__ bool tbf_group_u(const TBFArgs<T, R>& A, const TBLane& L, int32_t i, int32_t last,
                                            int32_t n_out, TBFRows& rw, TBFState<VEC, T, R>& S, R (&g32)[T],
                                            std::integer_sequence<int, Us...>)
{
    bool more = true;
    ((more = more && (i + Us <= last) ? (tbf_iter<VEC, T, UNIT, CHECK, Us>(A, L, i + Us, last, n_out, rw, S, g32),
                                         true)
                                      : false),
     ...);
    return more && i + (int)sizeof...(Us) <= last;
}

template <int VEC, int T, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tbf2d(TBFArgs<T, R> A)
{
    constexpr int H = tbf_halo(VEC, T);
    constexpr int W = (kWave - 2 * H) * VEC;
    constexpr int R0 = tbf_ring0(T);
    constexpr int WARM = (4 * T - 4 + R0 - 1) / R0;
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t ts = tl / (uint32_t)A.tiles_x;
    TBLane L;
    L.nx = (uint32_t)A.nx;
    L.ny = (int32_t)A.ny;
    L.row_bytes = L.nx * (uint32_t)sizeof(R);
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    L.voff = (uint32_t)wrap_row(x0, (int32_t)L.nx) * (uint32_t)sizeof(R);
    L.soff = (lane >= H && lane < kWave - H && x0 < (int32_t)L.nx) ? L.voff : kPastRow;
    const int32_t rows = (int32_t)A.rows;
    L.s0 = (int32_t)ts * rows;
    L.s1 = L.s0 + rows < L.ny ? L.s0 + rows : L.ny;
    L.dir = 1;
    L.yoff = 0;
    L.wrap_at = L.ny;
    L.wrap_to = 0;
    const int32_t n_out = L.s1 - L.s0;

    TBFState<VEC, T, R> S;
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
#pragma unroll
        for (int a = 0; a < R0; ++a) S.f0[a][j] = R(0);
#pragma unroll
        for (int a = 0; a < 2; ++a) S.p0[a][j] = S.mi[a][j] = R(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) S.wi[a][j] = R(0);
#pragma unroll
        for (int k = 0; k < T; ++k) {
#pragma unroll
            for (int a = 0; a < 8; ++a) S.fl[k][a][j] = R(0);
#pragma unroll
            for (int a = 0; a < 4; ++a) S.rw[k][a][j] = R(0);
#pragma unroll
            for (int a = 0; a < 2; ++a) S.pl[k][a][j] = S.rm[k][a][j] = R(0);
        }
    }

    // before iteration 0 (y = y0): phi^s rows y0-2 .. y0, phi_dot row y0-1,
    // w_in rows y0-T .. y0-T+2, mu_in row y0-T+1
    const int32_t y0 = L.s0 - 2 * T + 2;
    tb_load<VEC>(A.phi_s, wrap_row(y0 - 2, L.ny), L, L.row_bytes, S.f0[R0 - 2]);
    tb_load<VEC>(A.phi_s, wrap_row(y0 - 1, L.ny), L, L.row_bytes, S.f0[R0 - 1]);
    tb_load<VEC>(A.phi_s, wrap_row(y0, L.ny), L, L.row_bytes, S.f0[0]);
    tb_load<VEC>(A.pi_s, wrap_row(y0 - 1, L.ny), L, L.row_bytes, S.p0[1]);
    tb_load<VEC>(A.w_in, wrap_row(y0 - T, L.ny), L, L.row_bytes, S.wi[1]);
    tb_load<VEC>(A.w_in, wrap_row(y0 - T + 1, L.ny), L, L.row_bytes, S.wi[2]);
    tb_load<VEC>(A.w_in, wrap_row(y0 - T + 2, L.ny), L, L.row_bytes, S.wi[3]);
    tb_load<VEC>(A.mu_in, wrap_row(y0 - T + 1, L.ny), L, L.row_bytes, S.mi[1]);
    TBFRows rw;
    rw.phi = wrap_row(y0 + 1, L.ny);
    rw.pi = wrap_row(y0, L.ny);
    rw.w = wrap_row(y0 - T + 3, L.ny);
    rw.mu = wrap_row(y0 - T + 2, L.ny);

    R g32[T];
    double gs[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        g32[k] = R(0);
        gs[k] = 0.0;
    }
    const bool own_lane = L.soff != kPastRow;
    auto flush = [&]() {
#pragma unroll
        for (int k = 0; k < T; ++k) {
            gs[k] += own_lane ? (double)g32[k] : 0.0;
            g32[k] = R(0);
        }
    };

    const int32_t last = n_out + 4 * T - 5;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tbf_group_u<VEC, T, UNIT, true>(A, L, i, last, n_out, rw, S, g32,
                                                         std::make_integer_sequence<int, R0>{});
        i += R0;
    }
    flush();
    while (more) {
        more = tbf_group_u<VEC, T, UNIT, false>(A, L, i, last, n_out, rw, S, g32,
                                                std::make_integer_sequence<int, R0>{});
        i += R0;
        flush();
    }
    double gsum = 0.0;
#pragma unroll
    for (int k = 0; k < T; ++k) gsum += A.gscale[k] * wave_sum_f64(gs[k]);
    if (lane == 0) A.gacc[tile] += gsum;
}

// ----------------------------------------- T steps per HBM pass (3D) --------
//
// The 2D scheme with a second in-plane axis.  A wave marches along z; for
// every plane it holds NY = TY + 2T rows along y (rows y0-T .. y0+TY+T-1,
// periodic) of 64*VEC sites along x, with H = ceil(T/VEC) halo lanes per side
// as in 2D.  Level k (step n+k-1) is computed on the rows k .. NY-k-1 from
// level k-1 held in registers: y-neighbours are the adjacent register rows,
// x-neighbours DPP shifts, z-neighbours the planes of the pipelined march.
// Level T covers exactly the TY owned rows, the only ones written.  Rows of a
// ragged last tile beyond the lattice wrap around: they are computed but
// never stored.  A plane is addressed through one raw buffer descriptor
// spanning it (plane bytes < 2^31) and per-lane offsets of each register
// row, computed once per tile.

template <int T, typename R = float>
struct TB3Args {
    const R* phi_in;
    R* phi_out;
    const R* pi_in;
    R* pi_out;
    R* phi_lv[T];               // with ALL: phi^{n+k} of levels k = 1 .. T-1 (level T is phi_out)
    WavePartial* partials;
    int64_t nx, ny, nz;
    int64_t tiles_x, tiles_y, ntiles;
    int64_t rows;               // planes per tile along z
    int32_t zhalo = 0;          // 0: periodic in z; T: a z-slab stored with T halo planes below and above
    StepCoefT<R> k[T];
    DiagCoef dc;
};

template <int VEC, int T, int TY, typename R>
struct TB3State {
    static constexpr int NY = TY + 2 * T;
    R in[4][NY][VEC];           // phi^n planes, ring over the march
    R pin[2][NY][VEC];          // phi_dot^{n-1/2} planes (rows 1 .. NY-2)
    R lv[T][4][NY][VEC];        // level k planes (k = 1 .. T-1)
    R pl[T][2][NY][VEC];        // level k phi_dot planes
};

template <int T, int TY>
struct TB3Lane {
    static constexpr int NY = TY + 2 * T;
    uint32_t lrow[NY];          // byte offset in the plane of this lane's sites in register row r
    uint32_t srow[TY];          // the same for owned rows and lanes inside the lattice, else past the plane
    uint32_t plane_bytes;
    uint64_t plane;             // sites per plane
    int32_t nz;
    int32_t zwrap;              // plane count the march wraps at (none for a slab)
    int32_t zoff;               // stored plane of plane z is z + zoff (slab halo depth, else 0)
    int32_t s0, s1;             // output planes [s0, s1) of the tile
    int32_t yown;               // owned rows inside the lattice
    bool own_lane;
};

template <int VEC, int T, int TY, typename R>
__device__ __forceinline__ void tb3_load(const R* f, int32_t p, const TB3Lane<T, TY>& L, uint32_t bytes, int r0,
                                         int r1, R (&v)[TY + 2 * T][VEC])
{
    const R* base = f + (size_t)(uint32_t)p * L.plane;
#pragma unroll
    for (int r = 0; r < TY + 2 * T; ++r)
        if (r >= r0 && r < r1) buf_load<VEC>(base, bytes, L.lrow[r], v[r]);
}

// Iteration i of the z-march (z = s0 - T + 1 + i): level k computes plane
// s0 - T - k + 2 + i, as in 2D.
template <int VEC, int T, int TY, bool DIAG, bool UNIT, bool CHECK, int U, bool ALL, typename R>
__device__ __forceinline__ void tb3_iter(const TB3Args<T, R>& A, const TB3Lane<T, TY>& L, int32_t i, int32_t last,
                                         TBRows& rw, TB3State<VEC, T, TY, R>& S, DiagAcc& acc)
{
    constexpr int NY = TY + 2 * T;
    // prefetch phi^n plane z+2 and phi_dot plane z+1 (none after the last)
    const uint32_t nb = i < last ? L.plane_bytes : 0u;
    tb3_load<VEC, T, TY>(A.phi_in, rw.phi, L, nb, 0, NY, S.in[(U + 2) & 3]);
    tb3_load<VEC, T, TY>(A.pi_in, rw.pi, L, nb, 1, NY - 1, S.pin[(U + 1) & 1]);
    rw.phi = next_row(rw.phi, L.zwrap);
    rw.pi = next_row(rw.pi, L.zwrap);
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * (k - 1)) continue;
        const R(*cm)[VEC];
        const R(*cc)[VEC];
        const R(*cp)[VEC];
        const R(*pp)[VEC];
        if (k == 1) {
            cm = S.in[(U + 3) & 3];
            cc = S.in[U & 3];
            cp = S.in[(U + 1) & 3];
            pp = S.pin[U & 1];
        } else {
            cm = S.lv[k - 1][(U + 2) & 3];
            cc = S.lv[k - 1][(U + 3) & 3];
            cp = S.lv[k - 1][U & 3];
            pp = S.pl[k - 1][(U + 1) & 1];
        }
        // level 1 plane z is inside the tile for i in [T-1, T-1 + s1 - s0)
        const bool diag_plane = DIAG && k == 1 && i >= T - 1 && i < T - 1 + (L.s1 - L.s0);
        // level T plane s0 + i - (2T - 2), inside [s0, s1) once i >= 2T - 2
        const int32_t zout = L.s0 + i - (2 * T - 2);
        const uint32_t sb = (!CHECK || i >= 2 * T - 2) ? L.plane_bytes : 0u;
        const size_t obase = (size_t)(uint32_t)((CHECK && i < 2 * T - 2 ? L.s0 : zout) + L.zoff) * L.plane;
#pragma unroll
        for (int r = k; r < NY - k; ++r) {
            const R left = from_left_lane(cc[r][VEC - 1]);
            const R right = from_right_lane(cc[r][0]);
            R out_phi[VEC], out_pi[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const R c = cc[r][j];
                const R xm = j > 0 ? cc[r][j > 0 ? j - 1 : 0] : left;
                const R xp = j < VEC - 1 ? cc[r][j < VEC - 1 ? j + 1 : j] : right;
                kick_drift<3, UNIT>(c, nsum3(xm, xp, cc[r - 1][j], cc[r + 1][j], cm[r][j], cp[r][j]), pp[r][j],
                                    A.k[k - 1], out_pi[j], out_phi[j]);
                if constexpr (DIAG) {
                    if (k == 1 && r >= T && r < T + TY) {
                        if (diag_plane && r - T < L.yown && L.own_lane) {
                            const R nm[3] = {xm, cc[r - 1][j], cm[r][j]};
                            const R np[3] = {xp, cc[r + 1][j], cp[r][j]};
                            site_diag<3>(c, pp[r][j], nm, np, A.dc, acc);
                        }
                    }
                }
            }
            if (k < T) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    S.lv[k < T ? k : 0][U & 3][r][j] = out_phi[j];
                    S.pl[k < T ? k : 0][U & 1][r][j] = out_pi[j];
                }
                if constexpr (ALL) {
                    // owned rows of level k, plane s0 + i - (T + k - 2) when inside [s0, s1)
                    if (r >= T && r < T + TY) {
                        const int32_t e = i - (T + k - 2);
                        const bool in = e >= 0 && e < L.s1 - L.s0;
                        const size_t lb = (size_t)(uint32_t)((in ? L.s0 + e : L.s0) + L.zoff) * L.plane;
                        const uint32_t so = L.srow[r - T < TY ? (r - T >= 0 ? r - T : 0) : 0];
                        buf_store<VEC>(A.phi_lv[k < T ? k - 1 : 0] + lb, in ? L.plane_bytes : 0u, so, out_phi);
                    }
                }
            } else {
                const uint32_t so = L.srow[r - T < TY ? (r - T >= 0 ? r - T : 0) : 0];
                buf_store<VEC>(A.phi_out + obase, sb, so, out_phi);
                buf_store<VEC>(A.pi_out + obase, sb, so, out_pi);
            }
        }
    }
}

template <int VEC, int T, int TY, bool DIAG, bool UNIT, bool CHECK, bool ALL, typename R>
__device__ __forceinline__ bool tb3_group(const TB3Args<T, R>& A, const TB3Lane<T, TY>& L, int32_t i, int32_t last,
                                          TBRows& rw, TB3State<VEC, T, TY, R>& S, DiagAcc& acc)
{
    tb3_iter<VEC, T, TY, DIAG, UNIT, CHECK, 0, ALL>(A, L, i, last, rw, S, acc);
    if (i + 1 > last) return false;
    tb3_iter<VEC, T, TY, DIAG, UNIT, CHECK, 1, ALL>(A, L, i + 1, last, rw, S, acc);
    if (i + 2 > last) return false;
    tb3_iter<VEC, T, TY, DIAG, UNIT, CHECK, 2, ALL>(A, L, i + 2, last, rw, S, acc);
    if (i + 3 > last) return false;
    tb3_iter<VEC, T, TY, DIAG, UNIT, CHECK, 3, ALL>(A, L, i + 3, last, rw, S, acc);
    return i + 4 <= last;
}

// One wave's tile of a T-step 3D pass; `tile` must be below A.ntiles and
// wave-uniform.
template <int VEC, int T, int TY, bool DIAG, bool UNIT, bool ALL, typename R>
__device__ __forceinline__ void tb3_tile(const TB3Args<T, R>& A, int64_t tile)
{
    constexpr int H = (T + VEC - 1) / VEC;        // halo lanes per side
    constexpr int W = (kWave - 2 * H) * VEC;       // owned sites per wave along x
    constexpr int NY = TY + 2 * T;
    constexpr int WARM = (2 * T - 2 + 3) / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t rest = tl / (uint32_t)A.tiles_x;
    const uint32_t tyi = rest % (uint32_t)A.tiles_y;
    const uint32_t tz = rest / (uint32_t)A.tiles_y;
    const int32_t nx = (int32_t)A.nx, ny = (int32_t)A.ny;
    TB3Lane<T, TY> L;
    L.nz = (int32_t)A.nz;
    L.plane = (uint64_t)A.nx * (uint64_t)A.ny;
    L.plane_bytes = (uint32_t)(L.plane * sizeof(R));
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    const uint32_t xw = (uint32_t)wrap_row(x0, nx);
    L.own_lane = lane >= H && lane < kWave - H && x0 < nx;
    const int32_t y0 = (int32_t)tyi * TY;
    L.yown = ny - y0 < TY ? ny - y0 : TY;
#pragma unroll
    for (int r = 0; r < NY; ++r)
        L.lrow[r] = ((uint32_t)wrap_row(y0 - T + r, ny) * (uint32_t)nx + xw) * (uint32_t)sizeof(R);
#pragma unroll
    for (int r = 0; r < TY; ++r) L.srow[r] = (L.own_lane && r < L.yown) ? L.lrow[r + T] : kPastRow;
    const int32_t rows = (int32_t)A.rows;
    L.s0 = (int32_t)tz * rows;
    L.s1 = L.s0 + rows < L.nz ? L.s0 + rows : L.nz;
    // a slab reads its T halo planes instead of wrapping around
    L.zoff = A.zhalo;
    L.zwrap = L.nz + 2 * A.zhalo;   // stored planes: the wrap only ever meets loads of size 0 in a slab
    auto zplane = [&](int32_t z) { return A.zhalo ? z + A.zhalo : wrap_row(z, L.nz); };

    TB3State<VEC, T, TY, R> S;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < NY; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.in[a][r][j] = R(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.lv[k][a][r][j] = R(0);
            }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < NY; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.pin[a][r][j] = R(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.pl[k][a][r][j] = R(0);
            }

    // iteration 0 (z0 = s0 - T + 1) needs phi^n planes z0-1 .. z0+1 and phi_dot plane z0
    const int32_t z0 = L.s0 - T + 1;
    tb3_load<VEC, T, TY>(A.phi_in, zplane(z0 - 1), L, L.plane_bytes, 0, NY, S.in[3]);
    tb3_load<VEC, T, TY>(A.phi_in, zplane(z0), L, L.plane_bytes, 0, NY, S.in[0]);
    tb3_load<VEC, T, TY>(A.phi_in, zplane(z0 + 1), L, L.plane_bytes, 0, NY, S.in[1]);
    tb3_load<VEC, T, TY>(A.pi_in, zplane(z0), L, L.plane_bytes, 1, NY - 1, S.pin[0]);
    TBRows rw;
    rw.phi = zplane(z0 + 2);
    rw.pi = zplane(z0 + 1);

    DiagAcc acc;
    acc.links[0] = acc.links[1] = acc.links[2] = 0u;
    acc.walls = acc.nonfinite = 0u;
    acc.area = acc.ek = 0.0;

    const int32_t last = (L.s1 - L.s0) + 2 * T - 3;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tb3_group<VEC, T, TY, DIAG, UNIT, true, ALL>(A, L, i, last, rw, S, acc);
        i += 4;
    }
    while (more) {
        more = tb3_group<VEC, T, TY, DIAG, UNIT, false, ALL>(A, L, i, last, rw, S, acc);
        i += 4;
    }

    if constexpr (DIAG) {
        WavePartial w;
        w.links[0] = wave_sum_u32(acc.links[0]);
        w.links[1] = wave_sum_u32(acc.links[1]);
        w.links[2] = wave_sum_u32(acc.links[2]);
        w.walls = wave_sum_u32(acc.walls);
        w.nonfinite = wave_sum_u32(acc.nonfinite);
        w.pad = 0u;
        w.area = wave_sum_f64(acc.area);
        w.ek = wave_sum_f64(acc.ek);
        if (lane == 0) A.partials[tile] = w;
    }
}

template <int VEC, int T, int TY, bool DIAG, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tb3d(TB3Args<T, R> A)
{
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    tb3_tile<VEC, T, TY, DIAG, UNIT, false>(A, tile);
}

// The 3D T-step pass storing every step's field (adjoint recomputation).
template <int VEC, int T, int TY, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tb3d_all(TB3Args<T, R> A)
{
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    tb3_tile<VEC, T, TY, false, UNIT, true>(A, tile);
}

// ------------------ T steps per pass (3D) with LDS-shared row halos ---------
//
// The 3D pass of k_tb3d with a workgroup of NW waves stacked along y
// instead of independent waves: wave w holds R consecutive rows (workgroup
// rows w R .. w R + R - 1, of which the first and last T are the
// workgroup's halo) of 64 VEC sites along x for every level, and marches
// along z with the register plane rings of k_tb3d.  The y-neighbours of a
// wave's first and last row come from the waves next to it through LDS:
// after a wave computes a plane of level k it writes that plane's first and
// last row to LDS, and in the next iteration level k+1 reads the rows next
// to its own from there.  One barrier per iteration puts each plane's
// writes before its reads and its reads before the buffer is written again
// (two buffers per level, by plane parity).  The workgroup's NW R rows
// shrink by one per level at its edges, so level T is valid on the middle
// NW R - 2T rows, the only ones stored.  A wave holds R rows per level
// where k_tb3d holds R + 2T, and no row is computed twice inside a
// workgroup: the registers no longer bound the pass length, and the
// redundant work is 2T rows per NW R instead of per R.  NW is 8 or 16.

template <int VEC, int T, int R, typename RT>
struct TB3LState {
    RT in[4][R][VEC];           // phi^n planes, ring over the march
    RT pin[2][R][VEC];          // phi_dot^{n-1/2} planes
    RT lv[T][4][R][VEC];        // level k planes (k = 1 .. T-1)
    RT pl[T][2][R][VEC];        // level k phi_dot planes
};

template <int R>
struct TB3LLane {
    uint32_t lrow[R];           // byte offset in the plane of this lane's sites in each of the wave's rows
    uint32_t srow[R];           // the same for stored rows and owned lanes, else past the plane
    uint32_t plane_bytes;
    uint64_t plane;
    int32_t nz, zwrap, zoff;
    int32_t s0, s1;             // output planes [s0, s1) of the tile
    uint32_t own_rows;          // bit r: row r of this wave is stored (workgroup's middle rows, inside the lattice)
    bool own_lane;
    int wave;
};

// Rows R of one plane of field f at plane p for this wave.
template <int VEC, int R, typename RT>
__device__ __forceinline__ void tb3l_load(const RT* f, int32_t p, const TB3LLane<R>& L, uint32_t bytes,
                                          RT (&v)[R][VEC])
{
    const RT* base = f + (size_t)(uint32_t)p * L.plane;
#pragma unroll
    for (int r = 0; r < R; ++r) buf_load<VEC>(base, bytes, L.lrow[r], v[r]);
}

// LDS slot of (level k, plane parity, wave w, side 0 first row / 1 last row)
// for this lane.
template <int VEC, int NW, typename RT>
__device__ __forceinline__ RT* tb3l_slot(RT* lds, int k, int par, int w, int side)
{
    const int lane = threadIdx.x & (kWave - 1);
    return lds + ((((k * 2 + par) * NW + w) * 2 + side) * kWave + lane) * VEC;
}

template <int VEC, typename RT>
__device__ __forceinline__ void tb3l_put(RT* p, const RT (&v)[VEC])
{
#pragma unroll
    for (int j = 0; j < VEC; ++j) p[j] = v[j];
}

// Iteration i of the z-march (level k computes plane s0 - T - k + 2 + i, as
// in k_tb3d).
template <int VEC, int T, int R, int NW, bool DIAG, bool UNIT, bool CHECK, int U, bool ALL, typename RT>
__device__ __forceinline__ void tb3l_iter(const TB3Args<T, RT>& A, const TB3LLane<R>& L, RT* lds, int32_t i,
                                          int32_t last, TBRows& rw, TB3LState<VEC, T, R, RT>& S, DiagAcc& acc)
{
    // prefetch phi^n plane z+2 and phi_dot plane z+1 (none after the last)
    const uint32_t nb = i < last ? L.plane_bytes : 0u;
    tb3l_load<VEC, R>(A.phi_in, rw.phi, L, nb, S.in[(U + 2) & 3]);
    tb3l_load<VEC, R>(A.pi_in, rw.pi, L, nb, S.pin[(U + 1) & 1]);
    rw.phi = next_row(rw.phi, L.zwrap);
    rw.pi = next_row(rw.pi, L.zwrap);
    // the boundary rows of the phi^n plane level 1 computes next iteration
    tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, 0, U & 1, L.wave, 0), S.in[(U + 1) & 3][0]);
    tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, 0, U & 1, L.wave, 1), S.in[(U + 1) & 3][R - 1]);
    const int wb = L.wave > 0 ? L.wave - 1 : 0;
    const int wa = L.wave < NW - 1 ? L.wave + 1 : NW - 1;
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * (k - 1)) continue;
        const RT(*cm)[VEC];
        const RT(*cc)[VEC];
        const RT(*cp)[VEC];
        const RT(*pp)[VEC];
        if (k == 1) {
            cm = S.in[(U + 3) & 3];
            cc = S.in[U & 3];
            cp = S.in[(U + 1) & 3];
            pp = S.pin[U & 1];
        } else {
            cm = S.lv[k - 1][(U + 2) & 3];
            cc = S.lv[k - 1][(U + 3) & 3];
            cp = S.lv[k - 1][U & 3];
            pp = S.pl[k - 1][(U + 1) & 1];
        }
        // the rows next to this wave's first and last row in level k-1's
        // plane cc, written by the neighbouring waves last iteration (the
        // edge waves read their own rows: those results are never valid)
        RT yb[VEC], ya[VEC];
        {
            const RT* pb = tb3l_slot<VEC, NW>(lds, k - 1, (U + 1) & 1, wb, L.wave > 0 ? 1 : 0);
            const RT* pa = tb3l_slot<VEC, NW>(lds, k - 1, (U + 1) & 1, wa, L.wave < NW - 1 ? 0 : 1);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                yb[j] = pb[j];
                ya[j] = pa[j];
            }
        }
        const bool diag_plane = DIAG && k == 1 && i >= T - 1 && i < T - 1 + (L.s1 - L.s0);
        const int32_t zout = L.s0 + i - (2 * T - 2);
        const uint32_t sb = (!CHECK || i >= 2 * T - 2) ? L.plane_bytes : 0u;
        const size_t obase = (size_t)(uint32_t)((CHECK && i < 2 * T - 2 ? L.s0 : zout) + L.zoff) * L.plane;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const RT left = from_left_lane(cc[r][VEC - 1]);
            const RT right = from_right_lane(cc[r][0]);
            RT out_phi[VEC], out_pi[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const RT c = cc[r][j];
                const RT xm = j > 0 ? cc[r][j > 0 ? j - 1 : 0] : left;
                const RT xp = j < VEC - 1 ? cc[r][j < VEC - 1 ? j + 1 : j] : right;
                const RT ym = r > 0 ? cc[r > 0 ? r - 1 : 0][j] : yb[j];
                const RT yp = r < R - 1 ? cc[r < R - 1 ? r + 1 : r][j] : ya[j];
                kick_drift<3, UNIT>(c, nsum3(xm, xp, ym, yp, cm[r][j], cp[r][j]), pp[r][j], A.k[k - 1], out_pi[j],
                                    out_phi[j]);
                if constexpr (DIAG) {
                    if (k == 1 && diag_plane && ((L.own_rows >> r) & 1u) && L.own_lane) {
                        const RT nm[3] = {xm, ym, cm[r][j]};
                        const RT np[3] = {xp, yp, cp[r][j]};
                        site_diag<3>(c, pp[r][j], nm, np, A.dc, acc);
                    }
                }
            }
            if (k < T) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    S.lv[k < T ? k : 0][U & 3][r][j] = out_phi[j];
                    S.pl[k < T ? k : 0][U & 1][r][j] = out_pi[j];
                }
                if constexpr (ALL) {
                    // stored rows of level k, plane s0 + i - (T + k - 2) when inside [s0, s1)
                    const int32_t e = i - (T + k - 2);
                    const bool in = e >= 0 && e < L.s1 - L.s0;
                    const size_t lb = (size_t)(uint32_t)((in ? L.s0 + e : L.s0) + L.zoff) * L.plane;
                    buf_store<VEC>(A.phi_lv[k < T ? k - 1 : 0] + lb, in ? L.plane_bytes : 0u, L.srow[r], out_phi);
                }
            } else {
                buf_store<VEC>(A.phi_out + obase, sb, L.srow[r], out_phi);
                buf_store<VEC>(A.pi_out + obase, sb, L.srow[r], out_pi);
            }
        }
        if (k < T) {
            tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, k, U & 1, L.wave, 0), S.lv[k < T ? k : 0][U & 3][0]);
            tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, k, U & 1, L.wave, 1), S.lv[k < T ? k : 0][U & 3][R - 1]);
        }
    }
    __syncthreads();
}

template <int VEC, int T, int R, int NW, bool DIAG, bool UNIT, bool CHECK, bool ALL, typename RT>
__device__ __forceinline__ bool tb3l_group(const TB3Args<T, RT>& A, const TB3LLane<R>& L, RT* lds, int32_t i,
                                           int32_t last, TBRows& rw, TB3LState<VEC, T, R, RT>& S, DiagAcc& acc)
{
    tb3l_iter<VEC, T, R, NW, DIAG, UNIT, CHECK, 0, ALL>(A, L, lds, i, last, rw, S, acc);
    if (i + 1 > last) return false;
    tb3l_iter<VEC, T, R, NW, DIAG, UNIT, CHECK, 1, ALL>(A, L, lds, i + 1, last, rw, S, acc);
    if (i + 2 > last) return false;
    tb3l_iter<VEC, T, R, NW, DIAG, UNIT, CHECK, 2, ALL>(A, L, lds, i + 2, last, rw, S, acc);
    if (i + 3 > last) return false;
    tb3l_iter<VEC, T, R, NW, DIAG, UNIT, CHECK, 3, ALL>(A, L, lds, i + 3, last, rw, S, acc);
    return i + 4 <= last;
}

// Rows a workgroup of the LDS pass stores along y.
__host__ __device__ constexpr int tb3l_own_rows(int NW, int R, int T) { return NW * R - 2 * T; }

// Waves per SIMD the LDS pass leaves room for: a sixteen-wave workgroup
// needs four; with eight waves two workgroups per compute unit (four waves
// per SIMD) where the plane rings fit 128 registers without spilling, else
// one; diagnostic passes (one pass per record) take the registers they need.
constexpr int tb3l_min_waves(int vec, int T, int R, int NW, int esize, bool diag)
{
    return NW == 16 ? 4 : (!diag && esize == 4 && vec * R * (2 * T + 2) <= 48) ? 4 : 2;
}

// One workgroup's tile of the LDS pass; all its waves run the same march.
template <int VEC, int T, int R, int NW, bool DIAG, bool UNIT, bool ALL, typename RT>
__device__ __forceinline__ void tb3l_tile(const TB3Args<T, RT>& A, int64_t tile, RT* lds)
{
    constexpr int H = (T + VEC - 1) / VEC;
    constexpr int W = (kWave - 2 * H) * VEC;
    constexpr int YOWN = tb3l_own_rows(NW, R, T);
    constexpr int WARM = (2 * T - 2 + 3) / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t rest = tl / (uint32_t)A.tiles_x;
    const uint32_t tyi = rest % (uint32_t)A.tiles_y;
    const uint32_t tz = rest / (uint32_t)A.tiles_y;
    const int32_t nx = (int32_t)A.nx, ny = (int32_t)A.ny;
    TB3LLane<R> L;
    L.wave = wave_in_block();
    L.nz = (int32_t)A.nz;
    L.plane = (uint64_t)A.nx * (uint64_t)A.ny;
    L.plane_bytes = (uint32_t)(L.plane * sizeof(RT));
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    const uint32_t xw = (uint32_t)wrap_row(x0, nx);
    L.own_lane = lane >= H && lane < kWave - H && x0 < nx;
    const int32_t y0 = (int32_t)tyi * YOWN;          // first stored row of the workgroup
    L.own_rows = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t wr = L.wave * R + r - T;      // row relative to y0
        L.lrow[r] = ((uint32_t)wrap_row(y0 + wr, ny) * (uint32_t)nx + xw) * (uint32_t)sizeof(RT);
        const bool own = wr >= 0 && wr < YOWN && y0 + wr < ny;
        L.own_rows |= own ? (1u << r) : 0u;
        L.srow[r] = (own && L.own_lane) ? L.lrow[r] : kPastRow;
    }
    const int32_t rows = (int32_t)A.rows;
    L.s0 = (int32_t)tz * rows;
    L.s1 = L.s0 + rows < L.nz ? L.s0 + rows : L.nz;
    L.zoff = A.zhalo;
    L.zwrap = L.nz + 2 * A.zhalo;
    auto zplane = [&](int32_t z) { return A.zhalo ? z + A.zhalo : wrap_row(z, L.nz); };

    TB3LState<VEC, T, R, RT> S;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.in[a][r][j] = RT(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.lv[k][a][r][j] = RT(0);
            }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.pin[a][r][j] = RT(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.pl[k][a][r][j] = RT(0);
            }

    const int32_t z0 = L.s0 - T + 1;
    tb3l_load<VEC, R>(A.phi_in, zplane(z0 - 1), L, L.plane_bytes, S.in[3]);
    tb3l_load<VEC, R>(A.phi_in, zplane(z0), L, L.plane_bytes, S.in[0]);
    tb3l_load<VEC, R>(A.phi_in, zplane(z0 + 1), L, L.plane_bytes, S.in[1]);
    tb3l_load<VEC, R>(A.pi_in, zplane(z0), L, L.plane_bytes, S.pin[0]);
    TBRows rw;
    rw.phi = zplane(z0 + 2);
    rw.pi = zplane(z0 + 1);
    // level 1 of iteration 0 reads the boundary rows of plane z0 (parity 1)
    tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, 0, 1, L.wave, 0), S.in[0][0]);
    tb3l_put<VEC>(tb3l_slot<VEC, NW>(lds, 0, 1, L.wave, 1), S.in[0][R - 1]);
    __syncthreads();

    DiagAcc acc;
    acc.links[0] = acc.links[1] = acc.links[2] = 0u;
    acc.walls = acc.nonfinite = 0u;
    acc.area = acc.ek = 0.0;

    const int32_t last = (L.s1 - L.s0) + 2 * T - 3;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tb3l_group<VEC, T, R, NW, DIAG, UNIT, true, ALL>(A, L, lds, i, last, rw, S, acc);
        i += 4;
    }
    while (more) {
        more = tb3l_group<VEC, T, R, NW, DIAG, UNIT, false, ALL>(A, L, lds, i, last, rw, S, acc);
        i += 4;
    }

    if constexpr (DIAG) {
        WavePartial w;
        w.links[0] = wave_sum_u32(acc.links[0]);
        w.links[1] = wave_sum_u32(acc.links[1]);
        w.links[2] = wave_sum_u32(acc.links[2]);
        w.walls = wave_sum_u32(acc.walls);
        w.nonfinite = wave_sum_u32(acc.nonfinite);
        w.pad = 0u;
        w.area = wave_sum_f64(acc.area);
        w.ek = wave_sum_f64(acc.ek);
        if (lane == 0) A.partials[tile * NW + L.wave] = w;
    }
}

template <int VEC, int T, int R, int NW, bool DIAG, bool UNIT, bool ALL, typename RT>
__global__ __launch_bounds__(NW * kWave)
__attribute__((amdgpu_waves_per_eu(tb3l_min_waves(VEC, T, R, NW, (int)sizeof(RT), DIAG)))) void k_tb3l(TB3Args<T, RT> A)
{
    __shared__ RT lds[T * 2 * NW * 2 * kWave * VEC];
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x));
    if (tile >= A.ntiles) return;
    tb3l_tile<VEC, T, R, NW, DIAG, UNIT, ALL>(A, tile, lds);
}

// ------------------------------- reverse sweep, T steps per pass (3D) ------
//
// The 2D reverse pass (k_tba2d) on the 3D tile of k_tb3d: NY = TY + 2T rows
// along y per plane, level k (reverse step m-k+1) on rows k .. NY-k-1 with
// its own phi^{m-k+1} plane, w the stencil field and mu the pointwise one,
// separate in and out buffers, one dL/dV0 sum per level.

template <int T, typename R = float>
struct TBA3Args {
    const R* w_in;
    R* w_out;
    const R* mu_in;
    R* mu_out;
    const R* phi[T];
    double* gacc;
    int64_t nx, ny, nz;
    int64_t tiles_x, tiles_y, ntiles;
    int64_t rows;
    R a[T], b[T], cw[T], F[T];
    R kc, inv_dx2;
    double gscale[T];
};

template <int VEC, int T, int TY, typename R>
struct TBA3State {
    static constexpr int NY = TY + 2 * T;
    R in[4][NY][VEC];           // w planes
    R mi[2][NY][VEC];           // mu planes (rows 1 .. NY-2)
    R lv[T][4][NY][VEC];        // level k w planes
    R ml[T][2][NY][VEC];        // level k mu planes
    R ph[T][2][NY][VEC];        // phi plane of each level (rows k .. NY-k-1), one iteration ahead
};

template <int VEC, int T, int TY, bool UNIT, bool CHECK, int U, typename R>
__device__ __forceinline__ void tba3_iter(const TBA3Args<T, R>& A, const TB3Lane<T, TY>& L, int32_t i,
                                          int32_t last, TBRows& rw, int32_t (&prow)[T],
                                          TBA3State<VEC, T, TY, R>& S, double (&gs)[T])
{
    constexpr int NY = TY + 2 * T;
    const uint32_t nb = i < last ? L.plane_bytes : 0u;
    tb3_load<VEC, T, TY>(A.w_in, rw.phi, L, nb, 0, NY, S.in[(U + 2) & 3]);
    tb3_load<VEC, T, TY>(A.mu_in, rw.pi, L, nb, 1, NY - 1, S.mi[(U + 1) & 1]);
    rw.phi = next_row(rw.phi, L.nz);
    rw.pi = next_row(rw.pi, L.nz);
#pragma unroll
    for (int k = 0; k < T; ++k) {
        tb3_load<VEC, T, TY>(A.phi[k], prow[k], L, nb, k + 1, NY - k - 1, S.ph[k][(U + 1) & 1]);
        prow[k] = next_row(prow[k], L.nz);
    }
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (CHECK && i < 2 * (k - 1)) continue;
        const R(*cm)[VEC];
        const R(*cc)[VEC];
        const R(*cp)[VEC];
        const R(*mp)[VEC];
        if (k == 1) {
            cm = S.in[(U + 3) & 3];
            cc = S.in[U & 3];
            cp = S.in[(U + 1) & 3];
            mp = S.mi[U & 1];
        } else {
            cm = S.lv[k - 1][(U + 2) & 3];
            cc = S.lv[k - 1][(U + 3) & 3];
            cp = S.lv[k - 1][U & 3];
            mp = S.ml[k - 1][(U + 1) & 1];
        }
        const R(*ph)[VEC] = S.ph[k - 1][U & 1];
        const int32_t e = i - (T + k - 2);
        const bool own_plane = e >= 0 && e < L.s1 - L.s0;
        const int32_t zout = L.s0 + i - (2 * T - 2);
        const uint32_t sb = (!CHECK || i >= 2 * T - 2) ? L.plane_bytes : 0u;
        const size_t obase = (size_t)(uint32_t)(CHECK && i < 2 * T - 2 ? L.s0 : zout) * L.plane;
        double g = 0.0;
#pragma unroll
        for (int r = k; r < NY - k; ++r) {
            const R left = from_left_lane(cc[r][VEC - 1]);
            const R right = from_right_lane(cc[r][0]);
            R out_w[VEC], out_mu[VEC];
            double gr = 0.0;
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const R w = cc[r][j];
                const R xm = j > 0 ? cc[r][j > 0 ? j - 1 : 0] : left;
                const R xp = j < VEC - 1 ? cc[r][j < VEC - 1 ? j + 1 : j] : right;
                const R gp = adj_site<3, UNIT>(w, nsum3(xm, xp, cc[r - 1][j], cc[r + 1][j], cm[r][j], cp[r][j]),
                                               mp[r][j], ph[r][j], A.a[k - 1], A.b[k - 1], A.cw[k - 1], A.F[k - 1],
                                               A.kc, A.inv_dx2, out_w[j], out_mu[j]);
                gr += (double)gp;
            }
            // owned rows only (a wave-uniform factor: no per-lane select)
            if (r >= T && r < T + TY) g = fma(gr, r - T < L.yown ? 1.0 : 0.0, g);
            if (k < T) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    S.lv[k < T ? k : 0][U & 3][r][j] = out_w[j];
                    S.ml[k < T ? k : 0][U & 1][r][j] = out_mu[j];
                }
            } else {
                const uint32_t so = L.srow[r - T < TY ? (r - T >= 0 ? r - T : 0) : 0];
                buf_store<VEC>(A.w_out + obase, sb, so, out_w);
                buf_store<VEC>(A.mu_out + obase, sb, so, out_mu);
            }
        }
        if (own_plane) gs[k - 1] = fma(g, L.own_lane ? 1.0 : 0.0, gs[k - 1]);
    }
}

template <int VEC, int T, int TY, bool UNIT, bool CHECK, typename R>
__device__ __forceinline__ bool tba3_group(const TBA3Args<T, R>& A, const TB3Lane<T, TY>& L, int32_t i,
                                           int32_t last, TBRows& rw, int32_t (&prow)[T],
                                           TBA3State<VEC, T, TY, R>& S, double (&gs)[T])
{
    tba3_iter<VEC, T, TY, UNIT, CHECK, 0>(A, L, i, last, rw, prow, S, gs);
    if (i + 1 > last) return false;
    tba3_iter<VEC, T, TY, UNIT, CHECK, 1>(A, L, i + 1, last, rw, prow, S, gs);
    if (i + 2 > last) return false;
    tba3_iter<VEC, T, TY, UNIT, CHECK, 2>(A, L, i + 2, last, rw, prow, S, gs);
    if (i + 3 > last) return false;
    tba3_iter<VEC, T, TY, UNIT, CHECK, 3>(A, L, i + 3, last, rw, prow, S, gs);
    return i + 4 <= last;
}

template <int VEC, int T, int TY, bool UNIT, typename R>
__global__ __launch_bounds__(kBlock) void k_tba3d(TBA3Args<T, R> A)
{
    constexpr int H = (T + VEC - 1) / VEC;
    constexpr int W = (kWave - 2 * H) * VEC;
    constexpr int NY = TY + 2 * T;
    constexpr int WARM = (2 * T - 2 + 3) / 4;
    const int64_t tile = uniform64(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block());
    if (tile >= A.ntiles) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t tx = tl % (uint32_t)A.tiles_x;
    const uint32_t rest = tl / (uint32_t)A.tiles_x;
    const uint32_t tyi = rest % (uint32_t)A.tiles_y;
    const uint32_t tz = rest / (uint32_t)A.tiles_y;
    const int32_t nx = (int32_t)A.nx, ny = (int32_t)A.ny;
    TB3Lane<T, TY> L;
    L.nz = (int32_t)A.nz;
    L.plane = (uint64_t)A.nx * (uint64_t)A.ny;
    L.plane_bytes = (uint32_t)(L.plane * sizeof(R));
    const int32_t x0 = (int32_t)(tx * (uint32_t)W) + (lane - H) * VEC;
    const uint32_t xw = (uint32_t)wrap_row(x0, nx);
    L.own_lane = lane >= H && lane < kWave - H && x0 < nx;
    const int32_t y0 = (int32_t)tyi * TY;
    L.yown = ny - y0 < TY ? ny - y0 : TY;
#pragma unroll
    for (int r = 0; r < NY; ++r)
        L.lrow[r] = ((uint32_t)wrap_row(y0 - T + r, ny) * (uint32_t)nx + xw) * (uint32_t)sizeof(R);
#pragma unroll
    for (int r = 0; r < TY; ++r) L.srow[r] = (L.own_lane && r < L.yown) ? L.lrow[r + T] : kPastRow;
    const int32_t rows = (int32_t)A.rows;
    L.s0 = (int32_t)tz * rows;
    L.s1 = L.s0 + rows < L.nz ? L.s0 + rows : L.nz;

    TBA3State<VEC, T, TY, R> S;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < NY; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.in[a][r][j] = R(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.lv[k][a][r][j] = R(0);
            }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < NY; ++r)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                S.mi[a][r][j] = R(0);
#pragma unroll
                for (int k = 0; k < T; ++k) S.ml[k][a][r][j] = S.ph[k][a][r][j] = R(0);
            }

    const int32_t z0 = L.s0 - T + 1;
    tb3_load<VEC, T, TY>(A.w_in, wrap_row(z0 - 1, L.nz), L, L.plane_bytes, 0, NY, S.in[3]);
    tb3_load<VEC, T, TY>(A.w_in, wrap_row(z0, L.nz), L, L.plane_bytes, 0, NY, S.in[0]);
    tb3_load<VEC, T, TY>(A.w_in, wrap_row(z0 + 1, L.nz), L, L.plane_bytes, 0, NY, S.in[1]);
    tb3_load<VEC, T, TY>(A.mu_in, wrap_row(z0, L.nz), L, L.plane_bytes, 1, NY - 1, S.mi[0]);
    int32_t prow[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        tb3_load<VEC, T, TY>(A.phi[k], wrap_row(z0 - k, L.nz), L, L.plane_bytes, k + 1, NY - k - 1, S.ph[k][0]);
        prow[k] = wrap_row(z0 - k + 1, L.nz);
    }
    TBRows rw;
    rw.phi = wrap_row(z0 + 2, L.nz);
    rw.pi = wrap_row(z0 + 1, L.nz);
    double gs[T];
#pragma unroll
    for (int k = 0; k < T; ++k) gs[k] = 0.0;

    const int32_t last = (L.s1 - L.s0) + 2 * T - 3;
    int32_t i = 0;
    bool more = true;
#pragma unroll
    for (int w = 0; w < WARM; ++w) {
        if (more) more = tba3_group<VEC, T, TY, UNIT, true>(A, L, i, last, rw, prow, S, gs);
        i += 4;
    }
    while (more) {
        more = tba3_group<VEC, T, TY, UNIT, false>(A, L, i, last, rw, prow, S, gs);
        i += 4;
    }
    double gsum = 0.0;
#pragma unroll
    for (int k = 0; k < T; ++k) gsum += A.gscale[k] * wave_sum_f64(gs[k]);
    if (lane == 0) A.gacc[tile] += gsum;
}

// ------------------------------------------------------ launch templates --
//
// Host-side launchers for one field precision R; each kernel file
// instantiates them for its precision.  Coefficients arrive in FP64 and are
// rounded to R here, once per launch.

template <typename R>
StepCoefT<R> coef_as(const StepCoef64& k)
{
    StepCoefT<R> r;
    r.a = (R)k.a;
    r.b = (R)k.b;
    r.deta = (R)k.deta;
    r.F = (R)k.F;
    r.kc = (R)k.kc;
    r.inv_dx2 = (R)k.inv_dx2;
    return r;
}

template <typename R, int D, int VEC, int TY, bool UPDATE, bool DIAG>
hipError_t launch_t(const StepArgsT<R>& A, hipStream_t s)
{
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    // the plain update with dx = 1 and phi0 = 1 skips two exact
    // multiplications by 1 (same bits as the general form)
    if (UPDATE && !DIAG && A.k.inv_dx2 == R(1) && A.k.kc == R(1))
        hipLaunchKernelGGL((k_step<D, VEC, TY, UPDATE, DIAG, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0,
                           s, A);
    else
        hipLaunchKernelGGL((k_step<D, VEC, TY, UPDATE, DIAG, false, R>), dim3((unsigned)blocks), dim3(kBlock),
                           0, s, A);
    return hipGetLastError();
}

template <typename R, int D, int VEC, int TY>
hipError_t launch_mode(const StepArgsT<R>& A, bool update, bool diag, hipStream_t s)
{
    if (update && diag) return launch_t<R, D, VEC, TY, true, true>(A, s);
    if (update) return launch_t<R, D, VEC, TY, true, false>(A, s);
    if (diag) return launch_t<R, D, VEC, TY, false, true>(A, s);
    return hipSuccess;
}

template <typename R, int D, int VEC>
hipError_t launch_ty(const StepArgsT<R>& A, int ty, bool update, bool diag, hipStream_t s)
{
    if constexpr (D == 2) {
        return launch_mode<R, 2, VEC, 1>(A, update, diag, s);
    } else {
        switch (ty) {
        case 1: return launch_mode<R, 3, VEC, 1>(A, update, diag, s);
        case 2: return launch_mode<R, 3, VEC, 2>(A, update, diag, s);
        case 4: return launch_mode<R, 3, VEC, 4>(A, update, diag, s);
        default: return hipErrorInvalidValue;
        }
    }
}

// Lanes carry 16 bytes at most: VEC 1, 2, 4 in float32, VEC 1, 2 in float64.
template <typename R>
constexpr bool vec_ok(int vec)
{
    return vec == 1 || vec == 2 || (vec == 4 && sizeof(R) == 4);
}

template <typename R>
hipError_t launch_step_r(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                         void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s)
{
    const TileCounts c = tile_counts(g, t);
    StepArgsT<R> A;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_out);
    A.pi = static_cast<const R*>(pi);
    A.pi_out = static_cast<R*>(pi_out);
    A.partials = partials;
    A.nx = g.nx;
    A.Q = g.Q;
    A.M = g.M;
    A.tiles_x = c.tiles_x;
    A.tiles_q = c.tiles_q;
    A.ntiles = c.ntiles;
    A.rows = t.rows;
    A.k = coef_as<R>(k);
    A.dc = dc;
    if (g.ndim == 2) {
        switch (t.vec) {
        case 1: return launch_ty<R, 2, 1>(A, 1, update, diag, s);
        case 2: return launch_ty<R, 2, 2>(A, 1, update, diag, s);
        case 4:
            if constexpr (vec_ok<R>(4)) return launch_ty<R, 2, 4>(A, 1, update, diag, s);
            break;
        }
    } else {
        switch (t.vec) {
        case 1: return launch_ty<R, 3, 1>(A, step_ty(t.ty), update, diag, s);
        case 2: return launch_ty<R, 3, 2>(A, step_ty(t.ty), update, diag, s);
        case 4:
            if constexpr (vec_ok<R>(4)) return launch_ty<R, 3, 4>(A, step_ty(t.ty), update, diag, s);
            break;
        }
    }
    return hipErrorInvalidValue;
}

template <typename R, int D, int VEC, int TY>
hipError_t launch_adj_t(const AdjArgsT<R>& A, hipStream_t s)
{
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.inv_dx2 == R(1) && A.kc == R(1))
        hipLaunchKernelGGL((k_adjoint<D, VEC, TY, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_adjoint<D, VEC, TY, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R, int D, int VEC>
hipError_t launch_adj_ty(const AdjArgsT<R>& A, int ty, hipStream_t s)
{
    if constexpr (D == 2) {
        return launch_adj_t<R, 2, VEC, 1>(A, s);
    } else {
        switch (ty) {
        case 1: return launch_adj_t<R, 3, VEC, 1>(A, s);
        case 2: return launch_adj_t<R, 3, VEC, 2>(A, s);
        case 4: return launch_adj_t<R, 3, VEC, 4>(A, s);
        default: return hipErrorInvalidValue;
        }
    }
}

template <typename R>
hipError_t launch_adjoint_r(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                            const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s)
{
    const TileCounts tc = tile_counts(g, t);
    AdjArgsT<R> A;
    A.w_in = static_cast<const R*>(w_in);
    A.w_out = static_cast<R*>(w_out);
    A.mu = static_cast<R*>(mu);
    A.phi_n = static_cast<const R*>(phi_n);
    A.gacc = gacc;
    A.nx = g.nx;
    A.Q = g.Q;
    A.M = g.M;
    A.tiles_x = tc.tiles_x;
    A.tiles_q = tc.tiles_q;
    A.ntiles = tc.ntiles;
    A.rows = t.rows;
    A.a = (R)c.a;
    A.b = (R)c.b;
    A.cw = (R)c.cw;
    A.F = (R)c.F;
    A.kc = (R)c.kc;
    A.inv_dx2 = (R)c.inv_dx2;
    A.gscale = c.gscale;
    const int ty = g.ndim == 2 ? 1 : step_ty(t.ty);
    if (g.ndim == 2) {
        switch (t.vec) {
        case 1: return launch_adj_ty<R, 2, 1>(A, ty, s);
        case 2: return launch_adj_ty<R, 2, 2>(A, ty, s);
        case 4:
            if constexpr (vec_ok<R>(4)) return launch_adj_ty<R, 2, 4>(A, ty, s);
            break;
        }
    } else {
        switch (t.vec) {
        case 1: return launch_adj_ty<R, 3, 1>(A, ty, s);
        case 2: return launch_adj_ty<R, 3, 2>(A, ty, s);
        case 4:
            if constexpr (vec_ok<R>(4)) return launch_adj_ty<R, 3, 4>(A, ty, s);
            break;
        }
    }
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_adj_seed_r(const void* phi, int64_t count, double kc, double deta, void* mu, void* w,
                             double* partial, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_seed<R>), dim3(nblocks), dim3(kBlock), 0, s, static_cast<const R*>(phi), count,
                       (R)kc, (R)deta, static_cast<R*>(mu), static_cast<R*>(w), partial);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fill_r(void* phi, int64_t count, uint64_t seed, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_fill_uniform<R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, static_cast<R*>(phi),
                       count, seed);
    return hipGetLastError();
}

template <typename R, int VEC, int T>
hipError_t launch_tb_t(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi_in,
                       void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials, const DiagCoef& dc,
                       hipStream_t s, int yhalo = 0)
{
    TBArgs<T, R> A;
    A.yhalo = yhalo;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_out);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    A.partials = partials;
    A.nx = g.nx;
    A.ny = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.ntiles = A.tiles_x * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = dc;
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const bool unit = A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1);
    if (diag) {
        // float32 diagnostic passes also drop the unit factors (one VALU
        // instruction per site-update)
        if constexpr (sizeof(R) == 4) {
            if (unit) {
                hipLaunchKernelGGL((k_tb2d<VEC, T, true, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_tb2d<VEC, T, true, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    } else if (unit)
        hipLaunchKernelGGL((k_tb2d<VEC, T, false, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tb2d<VEC, T, false, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R, int VEC>
hipError_t launch_tb_v(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                       const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                       const DiagCoef& dc, hipStream_t s, int yhalo = 0)
{
    switch (T) {
    case 2: return launch_tb_t<R, VEC, 2>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
    case 3: return launch_tb_t<R, VEC, 3>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
    case 4: return launch_tb_t<R, VEC, 4>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
    case 6:
        if constexpr (sizeof(R) == 4 || VEC == 1)
            return launch_tb_t<R, VEC, 6>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
        break;
    case 8:
        if constexpr (sizeof(R) == 4 || VEC == 1)
            return launch_tb_t<R, VEC, 8>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
        break;
    }
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_tb3_all_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                            const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s);
template <typename R>
hipError_t launch_tba3_r(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                         const void* mu_in, void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c,
                         hipStream_t s);

// Multi-step passes of the adjoint (2D): the recomputation storing every
// step and the reverse sweep, T = 2, 4 and (float32) 8, vec 1 or 2.
template <typename R>
constexpr bool tba_combo_ok(int vec, int T)
{
    return (vec == 1 || vec == 2) && (T == 2 || T == 4 || (sizeof(R) == 4 && T == 8));
}

// The 2D recomputation follows the forward's multi-step passes: T = 2, 3, 4
// with vec 1, 2 and (float32) 4, and T = 6, 8 in float32 or with vec 1.
template <typename R>
constexpr bool tball_combo_ok(int vec, int T)
{
    return (vec == 1 || vec == 2 || (sizeof(R) == 4 && vec == 4)) &&
           (T == 2 || T == 3 || T == 4 || ((sizeof(R) == 4 || vec == 1) && (T == 6 || T == 8)));
}

// 2D forward passes with a kernel: T = 2, 3, 4 for every vec, T = 6, 8 in
// float32 or, in float64, with vec 1 (two sites of eight bytes per lane
// would need more than the register file).
template <typename R>
constexpr bool tb2_combo_ok(int vec, int T)
{
    return T == 2 || T == 3 || T == 4 || ((sizeof(R) == 4 || vec == 1) && (T == 6 || T == 8));
}

template <typename R, int VEC, int T>
hipError_t launch_tb_all_t(const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                           const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    TBArgs<T, R> A;
    A.yhalo = 0;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_lv[T - 1]);
    for (int i = 0; i < T; ++i) A.phi_lv[i] = static_cast<R*>(phi_lv[i]);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    A.partials = nullptr;
    A.nx = g.nx;
    A.ny = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.ntiles = A.tiles_x * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = DiagCoef{};
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1))
        hipLaunchKernelGGL((k_tb2d_all<VEC, T, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tb2d_all<VEC, T, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_tb_all_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                           const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    if (g.ndim == 3) return launch_tb3_all_r<R>(T, g, t, phi_in, phi_lv, pi_in, pi_out, k, s);
    if (!tball_combo_ok<R>(t.vec, T)) return hipErrorInvalidValue;
#define PRS_TBALL(V, TT)                                                                       \
    if (t.vec == V && T == TT) {                                                                \
        if constexpr (tball_combo_ok<R>(V, TT))                                                 \
            return launch_tb_all_t<R, V, TT>(g, t, phi_in, phi_lv, pi_in, pi_out, k, s);        \
    }
    PRS_TBALL(1, 2)
    PRS_TBALL(1, 3)
    PRS_TBALL(1, 4)
    PRS_TBALL(1, 6)
    PRS_TBALL(1, 8)
    PRS_TBALL(2, 2)
    PRS_TBALL(2, 3)
    PRS_TBALL(2, 4)
    PRS_TBALL(2, 6)
    PRS_TBALL(2, 8)
    PRS_TBALL(4, 2)
    PRS_TBALL(4, 3)
    PRS_TBALL(4, 4)
    PRS_TBALL(4, 6)
    PRS_TBALL(4, 8)
#undef PRS_TBALL
    return hipErrorInvalidValue;
}

template <typename R, int VEC, int T>
hipError_t launch_tba_t(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, const void* mu_in,
                        void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c, hipStream_t s)
{
    TBAArgs<T, R> A;
    A.w_in = static_cast<const R*>(w_in);
    A.w_out = static_cast<R*>(w_out);
    A.mu_in = static_cast<const R*>(mu_in);
    A.mu_out = static_cast<R*>(mu_out);
    for (int i = 0; i < T; ++i) {
        A.phi[i] = static_cast<const R*>(phi[i]);
        A.a[i] = (R)c[i].a;
        A.b[i] = (R)c[i].b;
        A.cw[i] = (R)c[i].cw;
        A.F[i] = (R)c[i].F;
        A.gscale[i] = c[i].gscale;
    }
    A.kc = (R)c[0].kc;
    A.inv_dx2 = (R)c[0].inv_dx2;
    A.gacc = gacc;
    A.nx = g.nx;
    A.ny = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.ntiles = A.tiles_x * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.inv_dx2 == R(1) && A.kc == R(1))
        hipLaunchKernelGGL((k_tba2d<VEC, T, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tba2d<VEC, T, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

// 2D T-step passes that also store the state after T/2 steps: T = 4, 6, 8
// where the forward pass has a kernel.
template <typename R, int VEC, int T>
hipError_t launch_tb_mid_t(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi_in,
                           void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k, hipStream_t s)
{
    TBArgs<T, R> A;
    A.yhalo = 0;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_out);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    for (int i = 0; i < T; ++i) A.phi_lv[i] = static_cast<R*>(phi_mid);
    A.pi_mid = static_cast<R*>(pi_mid);
    A.partials = nullptr;
    A.nx = g.nx;
    A.ny = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.ntiles = A.tiles_x * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = DiagCoef{};
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1))
        hipLaunchKernelGGL((k_tb2d_mid<VEC, T, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tb2d_mid<VEC, T, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R>
constexpr bool tbmid_combo_ok(int vec, int T)
{
    return (T == 4 || T == 6 || T == 8) && (vec == 1 || vec == 2 || (sizeof(R) == 4 && vec == 4)) &&
           (T == 4 || sizeof(R) == 4 || vec == 1);
}

template <typename R>
hipError_t launch_tb_mid_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                           const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                           hipStream_t s)
{
    if (g.ndim != 2 || t.ty != 1 || !tbmid_combo_ok<R>(t.vec, T)) return hipErrorInvalidValue;
#define PRS_TBMID(V, TT)                                                                                         \
    if (t.vec == V && T == TT) {                                                                                  \
        if constexpr (tbmid_combo_ok<R>(V, TT))                                                                   \
            return launch_tb_mid_t<R, V, TT>(g, t, phi_in, phi_out, pi_in, pi_out, phi_mid, pi_mid, k, s);      \
    }
    PRS_TBMID(1, 4)
    PRS_TBMID(1, 6)
    PRS_TBMID(1, 8)
    PRS_TBMID(2, 4)
    PRS_TBMID(2, 6)
    PRS_TBMID(2, 8)
    PRS_TBMID(4, 4)
    PRS_TBMID(4, 6)
    PRS_TBMID(4, 8)
#undef PRS_TBMID
    return hipErrorInvalidValue;
}

// The 2D reverse pass recomputing its fields (k_tbf2d): T = 2, 3, 4, vec 1
// or 2 in float32, vec 1 in float64 (the register rings of eight-byte
// values at two sites per lane would not fit).
template <typename R>
constexpr bool tbf_combo_ok(int vec, int T)
{
    return (vec == 1 || (sizeof(R) == 4 && vec == 2)) && (T == 2 || T == 3 || T == 4);
}

template <typename R, int VEC, int T>
hipError_t launch_tbf_t(const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s, const void* w_in,
                        void* w_out, const void* mu_in, void* mu_out, double* gacc, const StepCoef64* k,
                        const AdjCoef64* c, hipStream_t s)
{
    TBFArgs<T, R> A;
    A.phi_s = static_cast<const R*>(phi_s);
    A.pi_s = static_cast<const R*>(pi_s);
    A.w_in = static_cast<const R*>(w_in);
    A.w_out = static_cast<R*>(w_out);
    A.mu_in = static_cast<const R*>(mu_in);
    A.mu_out = static_cast<R*>(mu_out);
    for (int i = 0; i < T; ++i) {
        A.k[i] = coef_as<R>(k[i < T - 1 ? i : 0]);
        A.a[i] = (R)c[i].a;
        A.b[i] = (R)c[i].b;
        A.cw[i] = (R)c[i].cw;
        A.F[i] = (R)c[i].F;
        A.gscale[i] = c[i].gscale;
    }
    A.kc = (R)c[0].kc;
    A.inv_dx2 = (R)c[0].inv_dx2;
    A.gacc = gacc;
    A.nx = g.nx;
    A.ny = g.M;
    const int64_t W = (int64_t)(kWave - 2 * tbf_halo(VEC, T)) * VEC;
    A.tiles_x = (g.nx + W - 1) / W;
    A.ntiles = A.tiles_x * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    // the unit specialisation needs unit spacing and vacuum in both the
    // forward and the reverse coefficients (they come from the same run)
    if (A.inv_dx2 == R(1) && A.kc == R(1) && A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1))
        hipLaunchKernelGGL((k_tbf2d<VEC, T, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tbf2d<VEC, T, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_tbf_r(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                        const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                        const StepCoef64* k, const AdjCoef64* c, hipStream_t s)
{
    if (g.ndim != 2 || t.ty != 1 || !tbf_combo_ok<R>(t.vec, T)) return hipErrorInvalidValue;
#define PRS_TBF(V, TT)                                                                                  \
    if (t.vec == V && T == TT) {                                                                         \
        if constexpr (tbf_combo_ok<R>(V, TT))                                                            \
            return launch_tbf_t<R, V, TT>(g, t, phi_s, pi_s, w_in, w_out, mu_in, mu_out, gacc, k, c, s);   \
    }
    PRS_TBF(1, 2)
    PRS_TBF(1, 3)
    PRS_TBF(1, 4)
    PRS_TBF(2, 2)
    PRS_TBF(2, 3)
    PRS_TBF(2, 4)
#undef PRS_TBF
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_tba_r(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                        const void* mu_in, void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c,
                        hipStream_t s)
{
    if (g.ndim == 3) return launch_tba3_r<R>(T, g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);
    if (!tba_combo_ok<R>(t.vec, T)) return hipErrorInvalidValue;
#define PRS_TBA(V, TT)                                                                          \
    if (t.vec == V && T == TT) {                                                                 \
        if constexpr (tba_combo_ok<R>(V, TT))                                                    \
            return launch_tba_t<R, V, TT>(g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);    \
    }
    PRS_TBA(1, 2)
    PRS_TBA(1, 4)
    PRS_TBA(1, 8)
    PRS_TBA(2, 2)
    PRS_TBA(2, 4)
    PRS_TBA(2, 8)
#undef PRS_TBA
    return hipErrorInvalidValue;
}

// Owned rows per wave of a 3D multi-step pass for the tiling's ty (1, 2, 4:
// waves of their own; 8, 16: the LDS pass with 2 or 4 rows per wave, whose
// single steps and reverse steps run the kernels of ty 4).
__host__ __device__ __forceinline__ int tb3_rows(int ty)
{
    return ty == 4 ? 8 : 4;
}


// The LDS pass (k_tb3l): float32 vec 1 or 2 and float64 vec 1, 2 or 4 rows
// per wave, T = 2, 3, 4; sixteen-wave workgroups (whose waves must fit 128
// registers) with vec 1, or vec 2 and 2 rows per wave, in float32.
template <typename R>
constexpr bool tb3l_combo_ok(int vec, int T, int rows_per_wave, int nw = 8)
{
    if (nw == 16)
        return sizeof(R) == 4 && (T == 2 || T == 3 || T == 4) &&
               ((vec == 1 && (rows_per_wave == 2 || rows_per_wave == 4)) || (vec == 2 && rows_per_wave == 2));
    return nw == 8 && (T == 2 || T == 3 || T == 4) && (rows_per_wave == 2 || rows_per_wave == 4) &&
           (vec == 1 || (sizeof(R) == 4 && vec == 2));
}

// Waves and rows per wave of an LDS tiling: ty 8, 16 are eight waves of 2, 4
// rows; ty 32, 64 sixteen waves of 2, 4 rows.
__host__ __device__ __forceinline__ int tb3l_waves(int ty) { return ty >= 32 ? 16 : 8; }
__host__ __device__ __forceinline__ int tb3l_rows_per_wave(int ty) { return ty >= 32 ? ty / 16 : ty / 4; }

template <typename R, int VEC, int T, int RW, int NW>
hipError_t launch_tb3l_t(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi_in,
                         void* pi_out, void* const* phi_lv, const StepCoef64* k, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s, int zhalo = 0)
{
    TB3Args<T, R> A;
    A.zhalo = zhalo;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_out);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    for (int i = 0; i < T; ++i) A.phi_lv[i] = phi_lv ? static_cast<R*>(phi_lv[i]) : nullptr;
    A.partials = partials;
    A.nx = g.nx;
    A.ny = g.Q;
    A.nz = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    constexpr int YOWN = tb3l_own_rows(NW, RW, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.tiles_y = (g.Q + YOWN - 1) / YOWN;
    A.ntiles = A.tiles_x * A.tiles_y * ((g.M + t.rows - 1) / t.rows);   // workgroups
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = dc;
    const unsigned blocks = (unsigned)A.ntiles;
    const bool unit = A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1);
    if (phi_lv) {
        if (unit) hipLaunchKernelGGL((k_tb3l<VEC, T, RW, NW, false, true, true, R>), dim3(blocks), dim3(NW * kWave), 0, s, A);
        else hipLaunchKernelGGL((k_tb3l<VEC, T, RW, NW, false, false, true, R>), dim3(blocks), dim3(NW * kWave), 0, s, A);
    } else if (diag) {
        hipLaunchKernelGGL((k_tb3l<VEC, T, RW, NW, true, false, false, R>), dim3(blocks), dim3(NW * kWave), 0, s, A);
    } else if (unit) {
        hipLaunchKernelGGL((k_tb3l<VEC, T, RW, NW, false, true, false, R>), dim3(blocks), dim3(NW * kWave), 0, s, A);
    } else {
        hipLaunchKernelGGL((k_tb3l<VEC, T, RW, NW, false, false, false, R>), dim3(blocks), dim3(NW * kWave), 0, s, A);
    }
    return hipGetLastError();
}

// phi_lv non-NULL: the recomputation storing every step's field (phi_out is
// then phi_lv[T-1]).
template <typename R>
hipError_t launch_tb3l_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, void* const* phi_lv, const StepCoef64* k, bool diag,
                         WavePartial* partials, const DiagCoef& dc, hipStream_t s, int zhalo = 0)
{
    const int RW = tb3l_rows_per_wave(t.ty), NW = tb3l_waves(t.ty);
    if (!tb3l_tiling(t.ty) || !tb3l_combo_ok<R>(t.vec, T, RW, NW)) return hipErrorInvalidValue;
#define PRS_TB3L(V, TT, RR, WW)                                                                                 \
    if (t.vec == V && T == TT && RW == RR && NW == WW) {                                                         \
        if constexpr (tb3l_combo_ok<R>(V, TT, RR, WW))                                                           \
            return launch_tb3l_t<R, V, TT, RR, WW>(g, t, phi_in, phi_out, pi_in, pi_out, phi_lv, k, diag, partials, \
                                                   dc, s, zhalo);                                                \
    }
    PRS_TB3L(1, 2, 2, 8)
    PRS_TB3L(1, 3, 2, 8)
    PRS_TB3L(1, 4, 2, 8)
    PRS_TB3L(1, 2, 4, 8)
    PRS_TB3L(1, 3, 4, 8)
    PRS_TB3L(1, 4, 4, 8)
    PRS_TB3L(2, 2, 2, 8)
    PRS_TB3L(2, 3, 2, 8)
    PRS_TB3L(2, 4, 2, 8)
    PRS_TB3L(2, 2, 4, 8)
    PRS_TB3L(2, 3, 4, 8)
    PRS_TB3L(2, 4, 4, 8)
    PRS_TB3L(1, 2, 2, 16)
    PRS_TB3L(1, 3, 2, 16)
    PRS_TB3L(1, 4, 2, 16)
    PRS_TB3L(1, 2, 4, 16)
    PRS_TB3L(1, 3, 4, 16)
    PRS_TB3L(1, 4, 4, 16)
    PRS_TB3L(2, 2, 2, 16)
    PRS_TB3L(2, 3, 2, 16)
    PRS_TB3L(2, 4, 2, 16)
#undef PRS_TB3L
    return hipErrorInvalidValue;
}

template <typename R, int VEC, int T, int TY>
hipError_t launch_tb3_t(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi_in,
                        void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials, const DiagCoef& dc,
                        hipStream_t s, int zhalo = 0)
{
    TB3Args<T, R> A;
    A.zhalo = zhalo;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_out);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    A.partials = partials;
    A.nx = g.nx;
    A.ny = g.Q;
    A.nz = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.tiles_y = (g.Q + TY - 1) / TY;
    A.ntiles = A.tiles_x * A.tiles_y * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = dc;
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (diag)
        hipLaunchKernelGGL((k_tb3d<VEC, T, TY, true, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else if (A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1))
        hipLaunchKernelGGL((k_tb3d<VEC, T, TY, false, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tb3d<VEC, T, TY, false, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

// 3D multi-step passes: float32 T = 2, 3 with (vec 1, 4 or 8 rows) or
// (vec 2, 4 rows); float64 T = 2 with vec 1, 4 rows.
template <typename R>
constexpr bool tb3_combo_ok(int vec, int T, int TY)
{
    if (sizeof(R) == 8) return vec == 1 && T == 2 && TY == 4;
    return (T == 2 || T == 3) && ((vec == 1 && (TY == 4 || TY == 8)) || (vec == 2 && TY == 4));
}

// zhalo = T: the lattice is a z-slab stored with T halo planes below and
// above (plane z at z + T), which the march reads instead of wrapping.
template <typename R>
hipError_t launch_tb3d_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s, int zhalo = 0)
{
    if (tb3l_tiling(t.ty))
        return launch_tb3l_r<R>(T, g, t, phi_in, phi_out, pi_in, pi_out, nullptr, k, diag, partials, dc, s, zhalo);
    const int TY = tb3_rows(t.ty);
    if (!tb3_combo_ok<R>(t.vec, T, TY)) return hipErrorInvalidValue;
#define PRS_TB3(V, TT, YY)                                                                                   \
    if (t.vec == V && T == TT && TY == YY) {                                                                  \
        if constexpr (tb3_combo_ok<R>(V, TT, YY))                                                             \
            return launch_tb3_t<R, V, TT, YY>(g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, \
                                              zhalo);                                                         \
    }
    PRS_TB3(1, 2, 4)
    PRS_TB3(1, 2, 8)
    PRS_TB3(2, 2, 4)
    PRS_TB3(1, 3, 4)
    PRS_TB3(1, 3, 8)
    PRS_TB3(2, 3, 4)
#undef PRS_TB3
    return hipErrorInvalidValue;
}

// 3D multi-step passes of the adjoint: the recomputation on every 3D pass
// tiling (T = 2, 3); the reverse sweep with T = 2 on those tilings and, in
// float32, T = 3 with vec 1 and 4 rows (its register rows grow with T).
template <typename R>
constexpr bool tba3_combo_ok(int vec, int T, int TY)
{
    return (T == 2 && tb3_combo_ok<R>(vec, T, TY)) || (sizeof(R) == 4 && T == 3 && vec == 1 && TY == 4);
}

template <typename R, int VEC, int T, int TY>
hipError_t launch_tb3_all_t(const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                            const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    TB3Args<T, R> A;
    A.zhalo = 0;
    A.phi_in = static_cast<const R*>(phi_in);
    A.phi_out = static_cast<R*>(phi_lv[T - 1]);
    for (int i = 0; i < T; ++i) A.phi_lv[i] = static_cast<R*>(phi_lv[i]);
    A.pi_in = static_cast<const R*>(pi_in);
    A.pi_out = static_cast<R*>(pi_out);
    A.partials = nullptr;
    A.nx = g.nx;
    A.ny = g.Q;
    A.nz = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.tiles_y = (g.Q + TY - 1) / TY;
    A.ntiles = A.tiles_x * A.tiles_y * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    for (int i = 0; i < T; ++i) A.k[i] = coef_as<R>(k[i]);
    A.dc = DiagCoef{};
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.k[0].inv_dx2 == R(1) && A.k[0].kc == R(1))
        hipLaunchKernelGGL((k_tb3d_all<VEC, T, TY, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tb3d_all<VEC, T, TY, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R, int VEC, int T, int TY>
hipError_t launch_tba3_t(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, const void* mu_in,
                         void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c, hipStream_t s)
{
    TBA3Args<T, R> A;
    A.w_in = static_cast<const R*>(w_in);
    A.w_out = static_cast<R*>(w_out);
    A.mu_in = static_cast<const R*>(mu_in);
    A.mu_out = static_cast<R*>(mu_out);
    for (int i = 0; i < T; ++i) {
        A.phi[i] = static_cast<const R*>(phi[i]);
        A.a[i] = (R)c[i].a;
        A.b[i] = (R)c[i].b;
        A.cw[i] = (R)c[i].cw;
        A.F[i] = (R)c[i].F;
        A.gscale[i] = c[i].gscale;
    }
    A.kc = (R)c[0].kc;
    A.inv_dx2 = (R)c[0].inv_dx2;
    A.gacc = gacc;
    A.nx = g.nx;
    A.ny = g.Q;
    A.nz = g.M;
    const int64_t W = tb_owned_width_d(VEC, T);
    A.tiles_x = (g.nx + W - 1) / W;
    A.tiles_y = (g.Q + TY - 1) / TY;
    A.ntiles = A.tiles_x * A.tiles_y * ((g.M + t.rows - 1) / t.rows);
    A.rows = t.rows;
    const int64_t blocks = (A.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (A.inv_dx2 == R(1) && A.kc == R(1))
        hipLaunchKernelGGL((k_tba3d<VEC, T, TY, true, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    else
        hipLaunchKernelGGL((k_tba3d<VEC, T, TY, false, R>), dim3((unsigned)blocks), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_tb3_all_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                            const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s)
{
    if (tb3l_tiling(t.ty))
        return launch_tb3l_r<R>(T, g, t, phi_in, phi_lv[T - 1], pi_in, pi_out, phi_lv, k, false, nullptr, DiagCoef{},
                                s);
    const int TY = tb3_rows(t.ty);
    if (!tb3_combo_ok<R>(t.vec, T, TY)) return hipErrorInvalidValue;
#define PRS_TB3ALL(V, TT, YY)                                                                     \
    if (t.vec == V && T == TT && TY == YY) {                                                       \
        if constexpr (tb3_combo_ok<R>(V, TT, YY))                                                  \
            return launch_tb3_all_t<R, V, TT, YY>(g, t, phi_in, phi_lv, pi_in, pi_out, k, s);      \
    }
    PRS_TB3ALL(1, 2, 4)
    PRS_TB3ALL(1, 2, 8)
    PRS_TB3ALL(2, 2, 4)
    PRS_TB3ALL(1, 3, 4)
    PRS_TB3ALL(1, 3, 8)
    PRS_TB3ALL(2, 3, 4)
#undef PRS_TB3ALL
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_tba3_r(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                         const void* mu_in, void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c,
                         hipStream_t s)
{
    const int TY = tb3_rows(t.ty);
    if (!tba3_combo_ok<R>(t.vec, T, TY)) return hipErrorInvalidValue;
#define PRS_TBA3(V, TT, YY)                                                                             \
    if (t.vec == V && T == TT && TY == YY) {                                                             \
        if constexpr (tba3_combo_ok<R>(V, TT, YY))                                                       \
            return launch_tba3_t<R, V, TT, YY>(g, t, w_in, w_out, mu_in, mu_out, phi, gacc, c, s);       \
    }
    PRS_TBA3(1, 2, 4)
    PRS_TBA3(1, 2, 8)
    PRS_TBA3(2, 2, 4)
    PRS_TBA3(1, 3, 4)
#undef PRS_TBA3
    return hipErrorInvalidValue;
}

// yhalo = T: the lattice is a y-slab stored with T halo rows below and
// above (row y at y + T), which the march reads instead of wrapping.
template <typename R>
hipError_t launch_tb2d_r(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                         const DiagCoef& dc, hipStream_t s, int yhalo = 0)
{
    switch (t.vec) {
    case 1: return launch_tb_v<R, 1>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
    case 2: return launch_tb_v<R, 2>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
    case 4:
        if constexpr (vec_ok<R>(4))
            return launch_tb_v<R, 4>(T, g, t, phi_in, phi_out, pi_in, pi_out, k, diag, partials, dc, s, yhalo);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

}  // namespace prs
