// prs_ensemble.hip -- the batched ensemble's persistent kernel: many
// independent realisations (mixed 2D/3D lattices, sizes, eras, wall widths,
// time steps and step counts) advanced by one launch.
//
// Work.  Each realisation keeps its single-run pass plan (its tiling and
// steps per pass; no recorded state inside a pass; the diagnostics of a
// recorded state fused into the pass that starts there; a last
// diagnostics-only pass over the final state).  A pass is cut into work
// items: one to four wave tiles per wave of the workgroup's eight (2D
// multi-step passes and single steps), or one to four workgroup tiles of the
// 3D LDS-staged pass, and each tile runs the single-run code (tb_tile,
// tb3l_tile, step_tile), so a realisation's fields and records are bitwise
// those of the same realisation run alone.
//
// Order.  The realisations are dealt, longest first, onto a few sequences,
// each running its realisations' passes one after another; items are
// numbered round by round, round k holding the k-th pass of every sequence
// (with one sequence per realisation, round p is phase p: pass p of every
// realisation), optionally split into kEnsQueues queues with a contiguous
// slice of every pass each (one queue by default).  Workgroups take items
// from their queue's ticket counter.  An item of pass p waits until its own
// realisation has finished pass p - 1 (the fields it reads, and the buffers
// it overwrites, which pass p - 1 read); nothing waits for other
// realisations, so there is no grid barrier and a realisation's passes
// overlap the neighbouring phases of the others.  Every item an item waits
// for (an earlier pass of its realisation, in an earlier round) holds an
// earlier ticket, taken by a workgroup that is running, so the
// wait always ends whether or not the grid is co-resident; it is still
// bounded, and raises an error flag instead of hanging.
//
// Completion.  After an item its workgroup adds one to the realisation's
// arrival counter, once the item's stores are visible on every XCD: the
// multi-step passes store their fields with a device-coherent policy, so
// their items only wait for their stores; items that also store through the
// write-back L2 (records' partials, single steps) release it first (an L2
// write-back, which costs as much as a fifth of the run when done per item).
// The workgroup whose item completes a pass acquires, reduces that pass's
// record (one wave, finalize_wave, the single run's reduction) and publishes
// the pass as finished with a release; an item of the next pass acquires
// once its wait is over.

// The multi-step passes' field stores are device-coherent here (the SC1
// cache policy): a store completes only once it is visible to every XCD, so
// an item that stores nothing else can publish its arrival without writing
// back the XCD's L2 (see k_ens).
#define PRS_STORE_AUX 16

#include "prs_device.h"

namespace prs {

namespace {

constexpr int kEnsBlock = kEnsWaves * kWave;

// Most tiles per wave (workgroup tiles in 3D LDS passes) in one work item.
#ifndef PRS_ENS_MAX_CHUNK
#define PRS_ENS_MAX_CHUNK 4
#endif
constexpr int kEnsMaxChunk = PRS_ENS_MAX_CHUNK;

// The descriptors, pass tables and coefficients are read through the
// constant address space: they do not change during a launch, and loads
// from there are invariant, so the compiler may load a pass argument again
// where it is used instead of holding it in a register across the whole
// tile (the tiles of the eight-step pass need all their registers).
typedef const __attribute__((address_space(4))) EnsDesc CDesc;
typedef const __attribute__((address_space(4))) EnsPass CPass;
typedef const __attribute__((address_space(4))) EnsCoef CCoef;
// LDS of the 3D passes: vec 1, up to four steps, eight waves.
constexpr int kEnsLds = 4 * 2 * kEnsWaves * 2 * kWave;

__device__ __forceinline__ StepCoef ens_coef(CDesc& d, int64_t n)
{
    CCoef& c = ((CCoef*)d.coef)[n];
    StepCoef k;
    k.a = c.a;
    k.b = c.b;
    k.deta = d.deta;
    k.F = c.F;
    k.kc = d.kc;
    k.inv_dx2 = d.inv_dx2;
    return k;
}

__device__ __forceinline__ DiagCoef ens_diag(CDesc& d, int64_t n)
{
    DiagCoef dc;
    dc.V0 = ((CCoef*)d.coef)[n].dV0;
    dc.kc = d.dkc;
    return dc;
}

// A 2D T-step pass: one wave tile.
template <int VEC, int T, bool DIAG, bool UNIT>
__device__ __forceinline__ void ens_tb2(CDesc& d, CPass& ps, int64_t p, int64_t w)
{
    TBArgs<T> A;
    A.phi_in = d.phi[p & 1];
    A.phi_out = d.phi[(p + 1) & 1];
    A.pi_in = ps.alt ? d.pi_alt : d.pi;
    A.pi_out = ps.alt ? d.pi : d.pi_alt;
#pragma unroll
    for (int i = 0; i < T; ++i) A.phi_lv[i] = nullptr;
    A.pi_mid = nullptr;
    A.partials = DIAG ? d.part : nullptr;
    A.nx = d.nx;
    A.ny = d.M;
    A.tiles_x = ps.tiles_x;
    A.ntiles = ps.ntiles;
    A.rows = d.rows;
    A.yhalo = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) A.k[i] = ens_coef(d, ps.first + i);
    A.dc = ens_diag(d, ps.first);
    tb_tile<VEC, T, DIAG, UNIT>(A, w);
}

// A 3D T-step LDS-staged pass: one workgroup tile (every wave takes part).
template <int T, int R, bool DIAG, bool UNIT>
__device__ __forceinline__ void ens_tb3(CDesc& d, CPass& ps, int64_t p, int64_t tile, float* lds)
{
    TB3Args<T> A;
    A.phi_in = d.phi[p & 1];
    A.phi_out = d.phi[(p + 1) & 1];
    A.pi_in = ps.alt ? d.pi_alt : d.pi;
    A.pi_out = ps.alt ? d.pi : d.pi_alt;
#pragma unroll
    for (int i = 0; i < T; ++i) A.phi_lv[i] = nullptr;
    A.partials = DIAG ? d.part : nullptr;
    A.nx = d.nx;
    A.ny = d.Q;
    A.nz = d.M;
    A.tiles_x = ps.tiles_x;
    A.tiles_y = ps.tiles_q;
    A.ntiles = ps.ntiles;
    A.rows = d.rows;
    A.zhalo = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) A.k[i] = ens_coef(d, ps.first + i);
    A.dc = ens_diag(d, ps.first);
    tb3l_tile<1, T, R, kEnsWaves, DIAG, UNIT, false>(A, tile, lds);
}

// One step, or the diagnostics of the final state (UPDATE false): one wave tile.
template <int D, int VEC, bool UPDATE, bool DIAG, bool UNIT>
__device__ __forceinline__ void ens_step(CDesc& d, CPass& ps, int64_t p, int64_t w)
{
    StepArgs A;
    float* pin = ps.alt ? d.pi_alt : d.pi;
    A.phi_in = d.phi[p & 1];
    A.phi_out = d.phi[(p + 1) & 1];
    A.pi = pin;
    A.pi_out = pin;
    A.partials = DIAG ? d.part : nullptr;
    A.nx = d.nx;
    A.Q = d.Q;
    A.M = d.M;
    A.tiles_x = ps.tiles_x;
    A.tiles_q = ps.tiles_q;
    A.ntiles = ps.ntiles;
    A.rows = d.rows;
    A.k = ens_coef(d, UPDATE ? ps.first : 0);
    A.dc = ens_diag(d, ps.first);
    step_tile<D, VEC, 1, UPDATE, DIAG, UNIT>(A, w);
}

// The variants a single run launches for these settings (the plain update
// with dx = 1 and phi0 = 1 drops exact multiplications by 1; so do the
// float32 diagnostic passes in 2D).
template <int VEC, int T>
__device__ __forceinline__ void ens_tb2_mode(CDesc& d, CPass& ps, int64_t p, int64_t w, bool diag)
{
    if (diag) {
        if (d.unit) ens_tb2<VEC, T, true, true>(d, ps, p, w);
        else ens_tb2<VEC, T, true, false>(d, ps, p, w);
    } else {
        if (d.unit) ens_tb2<VEC, T, false, true>(d, ps, p, w);
        else ens_tb2<VEC, T, false, false>(d, ps, p, w);
    }
}

template <int T, int R>
__device__ __forceinline__ void ens_tb3_mode(CDesc& d, CPass& ps, int64_t p, int64_t tile,
                                             float* lds, bool diag)
{
    if (diag) ens_tb3<T, R, true, false>(d, ps, p, tile, lds);
    else if (d.unit) ens_tb3<T, R, false, true>(d, ps, p, tile, lds);
    else ens_tb3<T, R, false, false>(d, ps, p, tile, lds);
}

template <int D, int VEC>
__device__ __forceinline__ void ens_step_mode(CDesc& d, CPass& ps, int64_t p, int64_t w,
                                              bool update, bool diag)
{
    if (update && diag) ens_step<D, VEC, true, true, false>(d, ps, p, w);
    else if (update && d.unit) ens_step<D, VEC, true, false, true>(d, ps, p, w);
    else if (update) ens_step<D, VEC, true, false, false>(d, ps, p, w);
    else ens_step<D, VEC, false, true, false>(d, ps, p, w);
}

template <int VEC>
__device__ __forceinline__ void ens_tb2_len(CDesc& d, CPass& ps, int64_t p, int64_t w, bool diag)
{
    switch (ps.steps) {
    case 2: ens_tb2_mode<VEC, 2>(d, ps, p, w, diag); break;
    case 3: ens_tb2_mode<VEC, 3>(d, ps, p, w, diag); break;
    case 4: ens_tb2_mode<VEC, 4>(d, ps, p, w, diag); break;
    case 6:
        if constexpr (VEC <= 2) ens_tb2_mode<VEC, 6>(d, ps, p, w, diag);
        break;
    case 8:
        if constexpr (VEC <= 2) ens_tb2_mode<VEC, 8>(d, ps, p, w, diag);
        break;
    default: break;
    }
}

// Step c of item j of pass p.  Uniform across the workgroup.  A 3D LDS
// pass's item is ps.chunk consecutive workgroup tiles, one per step.  A 2D
// multi-step pass's item is a block of kEnsWaves row tiles (one per wave)
// by ps.chunk tile columns (one per step), so that the tiles above and below
// one another, which read each other's halo rows, run side by side and meet
// in L2.  A single step's item is ps.chunk runs of kEnsWaves consecutive
// wave tiles.
__device__ __forceinline__ void ens_tile(CDesc& d, CPass& ps, int64_t p, int64_t j, int c, float* lds)
{
    const bool diag = ps.rec >= 0;
    const int64_t t = j * ps.chunk + c;
    if (d.ndim == 3 && ps.steps > 1) {
        if (t >= ps.ntiles) return;
        if (d.ty == 8) {
            switch (ps.steps) {
            case 2: ens_tb3_mode<2, 2>(d, ps, p, t, lds, diag); break;
            case 3: ens_tb3_mode<3, 2>(d, ps, p, t, lds, diag); break;
            case 4: ens_tb3_mode<4, 2>(d, ps, p, t, lds, diag); break;
            default: break;
            }
        } else {
            switch (ps.steps) {
            case 2: ens_tb3_mode<2, 4>(d, ps, p, t, lds, diag); break;
            case 3: ens_tb3_mode<3, 4>(d, ps, p, t, lds, diag); break;
            default: break;
            }
        }
        return;
    }
    if (ps.steps > 1) {
        const int64_t by = j / ps.blocks_x, bx = j - by * ps.blocks_x;
        const int64_t ty = by * kEnsWaves + wave_in_block(), tx = bx * ps.chunk + c;
        if (tx >= ps.tiles_x || ty * ps.tiles_x >= ps.ntiles) return;
        const int64_t w = ty * ps.tiles_x + tx;
        switch (d.vec) {
        case 1: ens_tb2_len<1>(d, ps, p, w, diag); break;
        case 2: ens_tb2_len<2>(d, ps, p, w, diag); break;
        default: ens_tb2_len<4>(d, ps, p, w, diag); break;
        }
        return;
    }
    const int64_t w = t * kEnsWaves + wave_in_block();
    if (w >= ps.ntiles) return;
    const bool update = ps.steps == 1;
    if (d.ndim == 2) {
        switch (d.vec) {
        case 1: ens_step_mode<2, 1>(d, ps, p, w, update, diag); break;
        case 2: ens_step_mode<2, 2>(d, ps, p, w, update, diag); break;
        default: ens_step_mode<2, 4>(d, ps, p, w, update, diag); break;
        }
    } else {
        switch (d.vec) {
        case 1: ens_step_mode<3, 1>(d, ps, p, w, update, diag); break;
        case 2: ens_step_mode<3, 2>(d, ps, p, w, update, diag); break;
        default: ens_step_mode<3, 4>(d, ps, p, w, update, diag); break;
        }
    }
}

// Lane 0 waits until realisation r has finished `need` passes (relaxed
// polling; the caller acquires afterwards); false when the wait timed out
// (the error flag is then raised) or another wait already did.
__device__ __forceinline__ bool ens_wait(const EnsRun& E, int64_t r, uint32_t need)
{
    if (__hip_atomic_load(E.ready + r * kCtlStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(E.ready + r * kCtlStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (__hip_atomic_load(E.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (wall_clock64() - t0 > E.timeout) {
            __hip_atomic_store(E.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

typedef const __attribute__((address_space(4))) int64_t CI64;
typedef const __attribute__((address_space(4))) int32_t CI32;

// Wave 0: a ticket of queue q (lane 0 takes it; the value is uniform).
__device__ __forceinline__ uint32_t ens_ticket(const EnsRun& E, int q)
{
    uint32_t t = 0u;
    if ((threadIdx.x & (kWave - 1)) == 0)
        t = __hip_atomic_fetch_add(E.ticket + q * kCtlStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(t);
}

// Wave 0's position in its queue's tables: the phase and the phase entry of
// its last item.  A workgroup's tickets only grow, and so do the tables'
// starts, so the next item is found by moving forward from there.
struct EnsCursor {
    int32_t p, e;
};

// Wave 0: the last index in [from, to) whose start (a non-decreasing table
// read through `tab`) is at or below tk; tab[from] <= tk.  Sixty-four
// starts are read at once, one per lane, and counted with a ballot.
template <typename TAB>
__device__ __forceinline__ int32_t ens_seek(TAB* tab, int32_t from, int32_t to, int64_t tk)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        const int32_t idx = from + lane;
        const int64_t v = idx < to ? (int64_t)tab[idx] : INT64_MAX;
        const int32_t c = (int32_t)__builtin_popcountll(__ballot(v <= tk));
        if (c < kWave) return from + c - 1;
        from += kWave - 1;
    }
}

// Wave 0: ticket t of queue q as (realisation, pass, index), or realisation
// -1 when the launch has no such item or a wait failed; lane 0 waits.
// Queue q holds, round by round and sequence by sequence, items
// [q n / Q, (q+1) n / Q) of each pass of n items.
__device__ __forceinline__ void ens_decode(const EnsRun& E, int q, uint32_t t, EnsCursor& cur, int64_t& r,
                                           int64_t& p, int64_t& j)
{
    const int lane = threadIdx.x & (kWave - 1);
    r = -1;
    p = 0;
    j = 0;
    const int64_t* pstart = E.pstart + (int64_t)q * E.pstride;
    const int64_t* qstart = E.qstart + (int64_t)q * E.estride;
    CI32* off = (CI32*)E.phase_off;
    CI32* ent_r = (CI32*)E.ent_r;
    const int64_t tk = ((CI64*)pstart)[E.pb] + (int64_t)t;
    if (tk >= ((CI64*)pstart)[E.pe]) return;
    const int32_t ph = ens_seek(pstart, cur.p, E.pe, tk);
    const int32_t e0 = ph == cur.p ? cur.e : off[ph];
    const int32_t a = ens_seek(qstart, e0, off[ph + 1], tk);
    cur.p = ph;
    cur.e = a;
    const int64_t rr = ent_r[a];
    const int32_t pp = ((CI32*)E.ent_p)[a];
    const int64_t n = ((CPass*)((CDesc*)E.desc)[rr].passes)[pp].items;
    const int64_t j0 = __builtin_amdgcn_readfirstlane((int32_t)(tk - qstart[a]));
    uint32_t ok = 1u;
    if (lane == 0)
        ok = (__hip_atomic_load(E.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
              ens_wait(E, rr, (uint32_t)pp)) ? 1u : 0u;
    ok = __builtin_amdgcn_readfirstlane(ok);
    if (!ok) return;
    // the passes before this one, written on any XCD, become visible; the
    // invalidation completes before the barrier lets the other waves load
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    r = rr;
    p = pp;
    j = (int64_t)q * n / kEnsQueues + j0;
}

__global__ __launch_bounds__(kEnsBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_ens(EnsRun E)
{
    __shared__ float lds[kEnsLds];
    __shared__ int64_t s_item[3];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = wave_in_block();
    const int q = (int)(blockIdx.x % kEnsQueues);
    // wave 0 takes each item's successor while the item runs, so the
    // ticket's round trip overlaps the work
    uint32_t next = wave == 0 ? ens_ticket(E, q) : 0u;
    EnsCursor cur;
    cur.p = E.pb;
    cur.e = ((CI32*)E.phase_off)[E.pb];
    for (;;) {
        if (wave == 0) {
            int64_t r, p, j;
            ens_decode(E, q, next, cur, r, p, j);
            if (lane == 0) {
                s_item[0] = r;
                s_item[1] = p;
                s_item[2] = j;
            }
        }
        __syncthreads();
        const int64_t r = uniform64(s_item[0]);
        if (r < 0) break;
        const int64_t p = uniform64(s_item[1]);
        const int64_t j = uniform64(s_item[2]);
        if (wave == 0) next = ens_ticket(E, q);
        CDesc& d = ((CDesc*)E.desc)[r];
        CPass& ps = ((CPass*)d.passes)[p];
        const int chunk = ps.chunk;
        for (int c = 0; c < chunk; ++c) ens_tile(d, ps, p, j, c, lds);
        // every wave waits for its own stores of the item to reach L2 (the
        // barrier alone does not), so that wave 0's release covers them all
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (wave == 0) {
            uint32_t last = 0u;
            if (lane == 0) {
                // The item's stores must be visible on every XCD before its
                // arrival is.  A multi-step pass without diagnostics stores
                // only device-coherent fields, all complete by now (every
                // wave waited for them), so a relaxed arrival suffices; other
                // items (records' partials, single steps) also store through
                // the write-back L2, and release it first.
                const bool coherent = ps.steps > 1 && ps.rec < 0;
                const uint32_t old =
                    coherent ? __hip_atomic_fetch_add(E.arrive + r * kCtlStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : __hip_atomic_fetch_add(E.arrive + r * kCtlStride, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                last = (int64_t)old + 1 == ps.cum_end ? 1u : 0u;
            }
            last = __builtin_amdgcn_readfirstlane(last);
            if (last) {
                // every item's partials of the pass
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (ps.rec >= 0)
                    finalize_wave(d.part, ps.nparts, d.recs + ps.rec, ps.first,
                                  d.eta0 + (double)ps.first * d.deta64, d.area_scale);
                if (lane == 0)
                    __hip_atomic_store(E.ready + r * kCtlStride, (uint32_t)(p + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_ens_reset(uint32_t* __restrict__ v, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) v[i] = 0u;
}

}  // namespace

bool ens_supported(const Geometry& g, const Tiling& t, int T)
{
    if (g.f64 || !tiling_supported(g, t) || T < 1 || T > kMaxPassSteps) return false;
    if (T > 1 && !tb_supported(g)) return false;
    if (g.ndim == 2) return t.ty == 1 && (t.vec <= 2 || T <= 4);
    if (T == 1) return t.ty == 1 || ((t.ty == 8 || t.ty == 16) && t.vec == 1);
    return t.vec == 1 && ((t.ty == 8 && T <= 4) || (t.ty == 16 && T <= 3));
}

void ens_pass_grid(const Geometry& g, const Tiling& t, int L, EnsPass& ps)
{
    if (L > 1 && g.ndim == 3) {
        const int64_t W = tb_owned_width_d(1, L);
        const int64_t yown = tb3l_own_rows(kEnsWaves, t.ty / 4, L);
        const int64_t tx = (g.nx + W - 1) / W, tq = (g.Q + yown - 1) / yown;
        ps.tiles_x = (int32_t)tx;
        ps.tiles_q = (int32_t)tq;
        ps.ntiles = tx * tq * ((g.M + t.rows - 1) / t.rows);
        ps.nparts = ps.ntiles * kEnsWaves;
        ps.chunk = std::min(kEnsMaxChunk, ps.ntiles >= 1024 ? 4 : ps.ntiles >= 512 ? 2 : 1);
        ps.items = (int32_t)((ps.ntiles + ps.chunk - 1) / ps.chunk);
        return;
    }
    if (L > 1) {
        const int64_t W = tb_owned_width_d(t.vec, L);
        const int64_t tx = (g.nx + W - 1) / W;
        ps.tiles_x = (int32_t)tx;
        ps.tiles_q = 1;
        ps.ntiles = tx * ((g.M + t.rows - 1) / t.rows);
    } else {
        const TileCounts c = tile_counts(g, t);
        ps.tiles_x = (int32_t)c.tiles_x;
        ps.tiles_q = (int32_t)c.tiles_q;
        ps.ntiles = c.ntiles;
    }
    ps.nparts = ps.ntiles;
    // large passes hand out several tiles per wave at a time, so that the
    // cost of taking an item (a ticket, a lookup, an acquire) is spread over
    // more work; every pass still has many items
    ps.chunk = std::min(kEnsMaxChunk, ps.ntiles >= 8 * 4 * 64 ? 4 : ps.ntiles >= 8 * 2 * 64 ? 2 : 1);
    if (L > 1) {
        // blocks of kEnsWaves row tiles by chunk columns
        const int64_t rows_t = ps.ntiles / ps.tiles_x;
        ps.blocks_x = (int32_t)((ps.tiles_x + ps.chunk - 1) / ps.chunk);
        ps.items = (int32_t)(ps.blocks_x * ((rows_t + kEnsWaves - 1) / kEnsWaves));
    } else {
        ps.blocks_x = 0;
        ps.items = (int32_t)((ps.ntiles + kEnsWaves * ps.chunk - 1) / (kEnsWaves * ps.chunk));
    }
}

hipError_t ens_max_blocks(int* blocks)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ens, kEnsBlock, 0);
    if (e != hipSuccess) return e;
    *blocks = cus * (per > 0 ? per : 1);
    return hipSuccess;
}

hipError_t launch_ens_reset(uint32_t* ctl, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_ens_reset, dim3((unsigned)blocks), dim3(kBlock), 0, s, ctl, count);
    return hipGetLastError();
}

hipError_t launch_ens(const EnsRun& run, int blocks, hipStream_t s)
{
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ens, dim3((unsigned)blocks), dim3(kEnsBlock), 0, s, run);
    return hipGetLastError();
}

}  // namespace prs
