// Internal interface between the host API (prs_api.cpp) and the device code
// (prs_device.h, instantiated by prs_kernels.hip and prs_kernels_f64.hip).
// Not installed; the public contract is include/prs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "prs.h"

namespace prs {

// Per-step coefficients of Eqs. (4)-(6) from the FP64 schedule:
// a = (1-delta_n)/(1+delta_n), b = deta/(1+delta_n), F = 4 V0/phi0^2,
// kc = 1/phi0^2, so that the kick reads
// pi' = a pi + b (Lap phi - F phi (kc phi^2 - 1)).  The host computes them in
// FP64 (StepCoef64); a launch rounds them once to the field precision R.
template <typename R>
struct StepCoefT {
    R a, b, deta, F, kc, inv_dx2;
};
using StepCoef = StepCoefT<float>;
using StepCoef64 = StepCoefT<double>;

// FP64 constants of the diagnostics (Eq. 8 needs V(phi) = V0 (kc phi^2 - 1)^2).
struct DiagCoef {
    double V0, kc;
};

// Per-wave partial sums of one diagnostic pass; reduced in a fixed order.
struct WavePartial {
    uint32_t links[3];
    uint32_t walls;
    uint32_t nonfinite;
    uint32_t pad;
    double area;   // sum over crossing links of the Eq. (7) weight
    double ek;     // sum over wall sites of (1/2) phi_dot^2 / V
};

// Lattice seen by the kernels: x (fastest), a middle axis of Q rows (y in
// 3D, absent = 1 in 2D) and the marching axis of M planes (y in 2D, z in 3D).
struct Geometry {
    int ndim;
    int f64;    // 1: float64 fields, 0: float32
    int64_t nx, Q, M;
};

struct Tiling {
    int vec;    // sites per lane along x: 1, 2, 4
    int rows;   // planes per wave along the marching axis
    int ty;     // rows per wave along the middle axis (1 in 2D)
};

struct TileCounts {
    int64_t tiles_x, tiles_q, tiles_s, ntiles;
};

Geometry geometry_of(const prs_params& p);
TileCounts tile_counts(const Geometry& g, const Tiling& t);
bool tiling_supported(const Geometry& g, const Tiling& t);

// Field pointers below are device pointers to float32 or float64 values,
// as the Geometry says.

// One fused step over the whole lattice: reads phi_in and pi, writes
// phi_out and pi_out (pi_out == pi updates in place) when update; writes one
// WavePartial per wave tile when diag.  update == false && diag == true
// computes the diagnostics only.
hipError_t launch_step(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                       void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                       const DiagCoef& dc, hipStream_t s);

// T steps n .. n+T-1 in one pass (temporal blocking) with overlapped wave
// tiles; k holds the T step coefficients.  Reads phi_in and pi_in, writes
// phi^{n+T} to phi_out and phi_dot^{n+T-1/2} to pi_out (pi_out != pi_in).
// With diag, the partials are those of the input state.
hipError_t launch_tb(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                     const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                     const DiagCoef& dc, hipStream_t s);
// Number of wave tiles (and partials) of a T-step pass.
int64_t tb_tiles(const Geometry& g, const Tiling& t, int T);
// Multi-step passes exist for 2D lattices whose rows are shorter than 2^28
// sites and for 3D lattices whose planes are shorter than 2^31 bytes (their
// accesses use 32-bit byte offsets within a row or a plane).
bool tb_supported(const Geometry& g);
// Steps per multi-step pass with a kernel for some tiling: 2D 2, 3, 4, 6, 8;
// 3D 2 and, in float32, 3.
bool tb_steps_supported(const Geometry& g, int T);
// ... and for this tiling (2D float64: 6 and 8 with vec 1 only; 3D: vec 1
// or 2, and only some row counts).
bool tb_pass_supported(const Geometry& g, const Tiling& t, int T);
constexpr int kMaxPassSteps = 8;   // most leapfrog steps fused into one pass

// A T-step pass over a slab along the last axis (the per-device kernel of a
// lattice sharded along y in 2D, z in 3D): the fields are stored with T halo
// rows or planes below and above the g.M interior ones (row or plane z at
// z + T), read in place of the periodic wrap; only the interior rows or
// planes of phi_out and pi_out are written.  With diag, one WavePartial per
// wave tile (tb_tiles of them) of the input state's interior diagnostics.
hipError_t launch_tb_slab(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                          const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                          const DiagCoef& dc, hipStream_t s);
hipError_t launch_tb_slab_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                              const void* pi_in, void* pi_out, const StepCoef64* k, bool diag,
                              WavePartial* partials, const DiagCoef& dc, hipStream_t s);
hipError_t launch_tb_slab_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                              const void* pi_in, void* pi_out, const StepCoef64* k, bool diag,
                              WavePartial* partials, const DiagCoef& dc, hipStream_t s);

// Reduces `count` partials in a fixed order into one record at `rec`.
hipError_t launch_finalize(const WavePartial* partials, int64_t count, prs_stats* rec,
                           int64_t step, double eta, double area_scale, hipStream_t s);

hipError_t launch_fill_uniform(void* phi, int64_t count, uint64_t seed, bool f64, hipStream_t s);

// Coefficients of one reverse step n: a_n, b_n as in StepCoefT, cw = deta
// (0 on the final reverse step), gscale = -4 kc b_n.
template <typename R>
struct AdjCoefT {
    R a, b, cw, F, kc, inv_dx2;
    double gscale;
};
using AdjCoef64 = AdjCoefT<double>;

// One reverse step: reads w_in (with halo), mu and phi^n; writes w_out and mu
// (in place); adds this step's dL/dV0 contribution to gacc[wave tile].
hipError_t launch_adjoint(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                          const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s);

// Multi-step passes of the adjoint.  tb_all_supported: the recomputation
// (2D: as the forward passes, T = 2, 3, 4 and 6, 8 in float32 or with
// vec 1; 3D: as the forward passes); tba_supported: the reverse sweep (2D: T = 2, 4 and, in
// float32, 8, vec 1 or 2, ty 1; 3D: T = 2 on the 3D pass tilings and, in
// float32, T = 3 with vec 1, 4 rows).  launch_tb_all: T forward steps from (phi_in, pi_in) storing
// phi^{n+k} to phi_lv[k-1] for k = 1 .. T and phi_dot^{n+T-1/2} to pi_out
// (!= pi_in).  launch_tba: T reverse steps m, m-1, .. m-T+1 (coefficients
// c[k-1] and field phi[k-1] = phi^{m-k+1} for level k) from (w_in, mu_in) to
// (w_out, mu_out), both pairs distinct; adds the pass's dL/dV0 to
// gacc[wave tile] (tb_tiles(g, t, T) accumulators).
bool tba_supported(const Geometry& g, const Tiling& t, int T);
bool tb_all_supported(const Geometry& g, const Tiling& t, int T);
hipError_t launch_tb_all(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                         const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s);
hipError_t launch_tba(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out, const void* mu_in,
                      void* mu_out, const void* const* phi, double* gacc, const AdjCoef64* c, hipStream_t s);
hipError_t launch_tb_all_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                             const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s);
hipError_t launch_tb_all_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* const* phi_lv,
                             const void* pi_in, void* pi_out, const StepCoef64* k, hipStream_t s);
hipError_t launch_tba_f32(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                          const void* mu_in, void* mu_out, const void* const* phi, double* gacc,
                          const AdjCoef64* c, hipStream_t s);
hipError_t launch_tba_f64(int T, const Geometry& g, const Tiling& t, const void* w_in, void* w_out,
                          const void* mu_in, void* mu_out, const void* const* phi, double* gacc,
                          const AdjCoef64* c, hipStream_t s);

// Reverse passes that recompute their fields (2D): T reverse steps m .. s =
// m-T+1 from the pass-start state (phi_s = phi^s, pi_s = phi_dot^{s-1/2}),
// recomputing phi^{s+1} .. phi^{s+T-1} in registers with the forward
// coefficients k[0 .. T-2] (steps s .. s+T-2); c[k-1] and the adjoint
// buffers as for launch_tba.  tbf_supported: 2D, ty 1, T = 2, 3, 4, vec 1 or
// 2 (float64: vec 1).  tbf_tiles: wave tiles (and dL/dV0 accumulators) of
// such a pass.
// 2D T-step forward pass (T = 4, 6, 8) that also stores the state after T/2
// steps to (phi_mid, pi_mid).
bool tb_mid_supported(const Geometry& g, const Tiling& t, int T);
hipError_t launch_tb_mid(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                         const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                         hipStream_t s);
hipError_t launch_tb_mid_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                             const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                             hipStream_t s);
hipError_t launch_tb_mid_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                             const void* pi_in, void* pi_out, void* phi_mid, void* pi_mid, const StepCoef64* k,
                             hipStream_t s);
bool tbf_supported(const Geometry& g, const Tiling& t, int T);
int64_t tbf_tiles(const Geometry& g, const Tiling& t, int T);
int64_t tbf_workgroups(const Geometry& g, const Tiling& t, int T);   // of one launch
int64_t tb2_workgroups(const Geometry& g, const Tiling& t, int T);   // of one 2D T-step launch
hipError_t launch_tbf(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                      const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                      const StepCoef64* k, const AdjCoef64* c, hipStream_t s);
hipError_t launch_tbf_f32(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                          const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                          const StepCoef64* k, const AdjCoef64* c, hipStream_t s);
hipError_t launch_tbf_f64(int T, const Geometry& g, const Tiling& t, const void* phi_s, const void* pi_s,
                          const void* w_in, void* w_out, const void* mu_in, void* mu_out, double* gacc,
                          const StepCoef64* k, const AdjCoef64* c, hipStream_t s);

// mu = dL/dphi^S, w = deta*mu from the final field; FP64 loss partial per block.
hipError_t launch_adj_seed(const Geometry& g, const void* phi, int64_t count, double kc, double deta, void* mu,
                           void* w, double* partial, int nblocks, hipStream_t s);
hipError_t launch_sum_f64(const double* v, int64_t count, double* out, hipStream_t s);
// Statically allocated device scratch (4 MiB per device, resident for the
// life of the process): its device address on the current device and size.
// Every user on one device shares it.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
hipError_t static_scratch(void** ptr, size_t* bytes);

// Device copy of n16 16-byte words (16-byte aligned buffers).
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);
hipError_t launch_zero_f64(double* v, int64_t count, hipStream_t s);

// Per-precision instantiations behind the dispatchers above (one kernel file
// each).
hipError_t launch_step_f32(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                           void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s);
hipError_t launch_step_f64(const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out, const void* pi,
                           void* pi_out, const StepCoef64& k, bool update, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s);
hipError_t launch_tb_f32(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                           const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s);
hipError_t launch_tb_f64(int T, const Geometry& g, const Tiling& t, const void* phi_in, void* phi_out,
                           const void* pi_in, void* pi_out, const StepCoef64* k, bool diag, WavePartial* partials,
                           const DiagCoef& dc, hipStream_t s);
hipError_t launch_adjoint_f32(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                              const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s);
hipError_t launch_adjoint_f64(const Geometry& g, const Tiling& t, const void* w_in, void* w_out, void* mu,
                              const void* phi_n, double* gacc, const AdjCoef64& c, hipStream_t s);
hipError_t launch_adj_seed_f32(const void* phi, int64_t count, double kc, double deta, void* mu, void* w,
                               double* partial, int nblocks, hipStream_t s);
hipError_t launch_adj_seed_f64(const void* phi, int64_t count, double kc, double deta, void* mu, void* w,
                               double* partial, int nblocks, hipStream_t s);
hipError_t launch_fill_f32(void* phi, int64_t count, uint64_t seed, hipStream_t s);
hipError_t launch_fill_f64(void* phi, int64_t count, uint64_t seed, hipStream_t s);

// ---- batched ensemble: the persistent dataflow kernel (prs_ensemble.hip) ----
//
// Every realisation's single-run pass plan becomes a table of passes; each
// pass is cut into work items (eight wave tiles, or one workgroup tile of the
// LDS-staged 3D pass).  Items are numbered phase by phase (phase p holds pass
// p of every realisation that has one) and handed out by one ticket counter;
// an item of pass p waits until its own realisation has finished pass p-1.

// Per-step coefficients of one realisation: a_n, b_n and the force
// coefficient F_n rounded to float32 exactly as a single-run launch rounds
// them, and V0 a(eta_n)^beta of the diagnostics in FP64.
struct EnsCoef {
    float a, b, F, pad;
    double dV0;
};

struct EnsPass {
    int32_t first;      // first step n of the pass
    int32_t steps;      // 1 .. 8, or 0: diagnostics of the final state only
    int32_t rec;        // record index, or -1
    int32_t alt;        // 1: phi_dot is read from pi_alt
    int32_t tiles_x, tiles_q;   // tile grid of the pass (tiles_q: along y in 3D)
    int32_t items;      // work items of the pass
    int32_t chunk;      // tiles per wave (workgroup tiles in 3D multi-step passes) per item
    int32_t blocks_x;   // 2D multi-step passes: items along x (an item is kEnsWaves row tiles x chunk columns)
    int32_t pad;
    int64_t ntiles;     // wave tiles, or workgroup tiles of a 3D multi-step pass
    int64_t nparts;     // wave partials the record reduces
    int64_t cum_end;    // items of this realisation's passes up to this one
};

struct EnsDesc {
    float* phi[2];      // pass p reads phi[p & 1] and writes phi[(p + 1) & 1]
    float* pi;          // the caller's phi_dot
    float* pi_alt;      // second phi_dot field of multi-step passes
    const EnsCoef* coef;
    const EnsPass* passes;
    WavePartial* part;
    prs_stats* recs;
    int64_t nx, Q, M;
    int32_t ndim, vec, ty, rows;
    int32_t npasses, unit;      // unit: dx = 1 and phi0 = 1
    float deta, kc, inv_dx2, pad;
    double eta0, deta64, area_scale, dkc;
};

// Work queues of the ensemble kernel: workgroup b takes its items from queue
// b % kEnsQueues, each queue holding a contiguous slice of every pass.  One
// queue per XCD (eight, so that neighbouring tiles meet in one L2) measured
// 4 % slower than a single queue on the 64-member ensemble: a pass then
// completes only when the slowest of its eight slices does.  Correctness
// does not depend on the number of queues nor on where a workgroup runs.
#ifndef PRS_ENS_QUEUES
#define PRS_ENS_QUEUES 1
#endif
constexpr int kEnsQueues = PRS_ENS_QUEUES;

// Sequences the one-launch ensemble deals its realisations onto (0: one per
// realisation, i.e. phase order: pass p of every realisation, then pass
// p + 1).  A sequence runs its realisations' passes one after another and
// the tickets take the sequences' passes in turn, so only about this many
// realisations are in flight at a time.
#ifndef PRS_ENS_SEQUENCES
#define PRS_ENS_SEQUENCES 16
#endif
constexpr int kEnsSequences = PRS_ENS_SEQUENCES;

// Distance in 32-bit words between the ensemble kernel's counters: one
// 128-byte cache line each, so that atomics on different counters (the
// tickets, each realisation's arrivals and finished passes) never queue
// behind one another on a shared line.
constexpr int kCtlStride = 32;

struct EnsRun {
    const EnsDesc* desc;
    const int64_t* pstart;          // [queue][phase]: items of the queue before each phase (pstride per queue)
    const int32_t* phase_off;       // nphase + 1 offsets into the round entries
    const int32_t* ent_r;           // realisation of each round entry
    const int32_t* ent_p;           // its pass
    const int64_t* qstart;          // [queue][entry]: first item of the entry's slice in the queue (estride per queue)
    uint32_t* ticket;               // kEnsQueues ticket counters of this launch (kCtlStride apart)
    uint32_t* arrive;               // per realisation: items finished (kCtlStride apart)
    uint32_t* ready;                // per realisation: passes finished (kCtlStride apart)
    int32_t* err;                   // raised when a wait times out
    int64_t pstride, estride;
    int32_t pb, pe;                 // phases [pb, pe) of this launch
    uint64_t timeout;               // wall-clock ticks a wait may take
};

// Waves per workgroup of the ensemble kernel.
constexpr int kEnsWaves = 8;

// Settings the ensemble kernel holds code for (float32): 2D ty 1 with vec 1
// or 2 and T <= 8, or vec 4 and T <= 4; 3D single steps (T = 1) with ty 1 and
// vec 1, 2 or 4; 3D LDS-staged passes with vec 1 and ty 8 (T <= 4) or ty 16
// (T <= 3).
bool ens_supported(const Geometry& g, const Tiling& t, int T);
// Wave tiles, tile grid and items of one pass of length L (0: diagnostics only).
void ens_pass_grid(const Geometry& g, const Tiling& t, int L, EnsPass& ps);
hipError_t ens_max_blocks(int* blocks);
hipError_t batch_clock_rate_khz(int* khz);
// Zeroes `count` 32-bit counters (a kernel, so that it can be captured).
hipError_t launch_ens_reset(uint32_t* ctl, int64_t count, hipStream_t s);
hipError_t launch_ens(const EnsRun& run, int blocks, hipStream_t s);
hipError_t launch_zero_f32(float* v, int64_t count, hipStream_t s);

}  // namespace prs
