// HIP kernels (gfx950, wave64) of the lattice Boltzmann - immersed boundary
// capsule solver (arXiv:1903.03356).
//
// Grid kernel: one fused pass per time step.  It pulls the nine populations
// (streaming, Eq. 1 left side), applies the Zou-He walls (Sec. 2.1), takes the
// force-corrected moments (Eqs. 6-7) and writes the BGK collision with the
// forcing term (Eqs. 2, 4, 5).  Populations are stored as deviations
// f_i - w_i, structure of arrays [9][ny][nxp], x fastest.  The stored buffer
// holds post-collision values; the next pass pulls them.
//
// IB kernel: one workgroup per capsule.  It stages the moments of the
// capsule's fluid patch in LDS and runs the Lagrangian part of the step
// (Secs. 2.2-2.4).  It spreads the force with 64-bit fixed-point atomics, so
// the force field is bit-reproducible.
#include "lbib_device.h"

#include <hip/hip_ext.h>

#include <math.h>

namespace lbib {

// ------------------------------------------------------------ grid kernel
// Population stores: streaming (non-temporal) writes.  Each value is read
// once, by the next step, so keeping it in L2 buys nothing, and the dirty lines
// it would leave there lengthen the write-back at the end of every launch.
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Population store: streaming (NT) or plain.  A lattice whose two population
// buffers fit in the memory-side cache (256 MB on MI355X) keeps them there
// with plain stores, and the next step reads them from it (single pass,
// measured: 1024^2 15.5 -> 13.8 us, 1448^2 29.8 -> 25.5 us, 2048^2 53.8 ->
// 52.5 us; 2896^2 105.6 -> 111.9 us and 4096^2 203.5 -> 210.8 us the other way).
template <typename T, bool NT>
__device__ __forceinline__ void put_pop(T* p, T v)
{
    if (NT) st_stream(p, v);
    else *p = v;
}

// One lattice node with total force (Fx, Fy), from its pulled and completed
// populations s: force-corrected moments, BGK + forcing, store.
template <typename T, bool NT = true>
__device__ __forceinline__ void collide_pulled(const T (&s)[9], T* __restrict__ dst,
                                               const GridArgs& g, int x, int y, T Fx, T Fy)
{
    const size_t cell = (size_t)y * g.nxp + x;
    const T drho = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])) + s[8];
    const T rho = T(1) + drho;
    const T jx = (s[1] - s[3]) + (s[5] - s[6]) + (s[8] - s[7]);
    const T jy = (s[2] - s[4]) + (s[5] + s[6]) - (s[7] + s[8]);
    const T irho = T(1) / rho;
    // rho u (Eq. 7): mx = rho u_x - u_ref(y) is the momentum the stored values carry
    const T mx = jx + T(0.5) * Fx, my = jy + T(0.5) * Fy;
    const T ux = (uref_at<T>(g, y) + mx) * irho, uy = my * irho;
    const T om = (T)g.omega;
    const T pre = T(1) - T(0.5) * om;
    const T usq15 = T(1.5) * (ux * ux + uy * uy);
    const T uF = ux * Fx + uy * Fy;
    const T wa = T(1.0 / 9.0), wd = T(1.0 / 36.0);
    const T w3a = FirstOrderW<T>::axis, w3d = FirstOrderW<T>::diag;
    const size_t plane = (size_t)g.ny * g.nxp;
    T* o = dst + cell;
    put_pop<T, NT>(&o[0], relax(s[0], T(4.0 / 9.0), T(0), T(0), T(0), T(0), drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[plane], relax(s[1], wa, w3a, ux, mx, Fx, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[2 * plane], relax(s[2], wa, w3a, uy, my, Fy, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[3 * plane], relax(s[3], wa, w3a, -ux, -mx, -Fx, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[4 * plane], relax(s[4], wa, w3a, -uy, -my, -Fy, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[5 * plane], relax(s[5], wd, w3d, ux + uy, mx + my, Fx + Fy, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[6 * plane], relax(s[6], wd, w3d, uy - ux, my - mx, Fy - Fx, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[7 * plane], relax(s[7], wd, w3d, -ux - uy, -mx - my, -Fx - Fy, drho, rho, usq15, uF, om, pre));
    put_pop<T, NT>(&o[8 * plane], relax(s[8], wd, w3d, ux - uy, mx - my, Fx - Fy, drho, rho, usq15, uF, om, pre));
}

// One lattice node with the IB force of this step.  A wave holds one 64-cell
// row segment (y and seg are the same in all its lanes).  The wave also clears
// the force accumulator of the previous time level in its segment (if that
// segment was active), so the next IB launch finds it zeroed; each segment has
// exactly one owning wave, which reads its two activity flags before clearing
// one.
//
// The nine population loads go out together with the segment's flags (and,
// for the far part of a split step, FAR, its near-map entry), and the wave
// waits for all of them once: the populations do not depend on the flags.
// (Issued after the flags, they would wait for the flags' round trip first.)
// The far part skips a segment whose near-map entry carries this step's stamp
// (the near pass computes it) and raises ST_NEAR where it finds an active
// force flag: the near regions were too small.
template <bool OPEN, bool NT = true, bool FAR = false, typename T>
__device__ __forceinline__ void grid_cell(const T* __restrict__ src, T* __restrict__ dst,
                                          const long long* __restrict__ fib_now,
                                          const int* __restrict__ flags_now,
                                          long long* __restrict__ fib_old,
                                          int* __restrict__ flags_old, const GridArgs& g, int y,
                                          int seg, int lane, const int* __restrict__ near_map = nullptr,
                                          int stamp = 0, int* status = nullptr)
{
    const int x = seg * kSegW + lane;
    const int fidx = y * g.nseg + seg;
    const size_t cell = (size_t)y * g.nxp + x;
    const bool in = x < g.nx;
    // lanes past the row's end (x < nxp) load the last node's values and
    // store nothing
    T s[9];
    pull_loads<T, OPEN>(src, in ? x : g.nx - 1, y, g, s);
    const int act = flags_now[fidx];
    const int old = flags_old[fidx];
    const int mark = FAR ? near_map[fidx] : 0;
    // keep these loads here, ahead of the branches on the flags (otherwise
    // they may be moved into the branches that use them, one round trip each)
#pragma unroll
    for (int i = 0; i < 9; i++) asm volatile("" ::"v"(s[i]));
    asm volatile("" ::"v"(act), "v"(old), "v"(mark));
    if (FAR) {
        if (mark == stamp) return;
        if ((act | old) && lane == 0) atomicOr(status, ST_NEAR);
    }
    if (in) {
        T Fx = (T)g.gx, Fy = T(0);
        if (act) {
            const longlong2 f = *reinterpret_cast<const longlong2*>(fib_now + 2 * cell);
            Fx += fix_to_real<T>(f.x);
            Fy += fix_to_real<T>(f.y);
        }
        pull_complete<T, OPEN>(src, x, y, g, Fx, s);
        collide_pulled<T, NT>(s, dst, g, x, y, Fx, Fy);
    }
    if (old) {
        *reinterpret_cast<longlong2*>(fib_old + 2 * cell) = make_longlong2(0, 0);
        if (lane == 0) flags_old[fidx] = 0;
    }
}

// ---- near / far split of a grid step (IB launch hidden behind the far part)
// Rows and 64-cell segments of a capsule's near region (rect in world cells,
// x unwrapped).  The IB kernel stamps exactly these (row, segment) units into
// the near map and the near kernel computes exactly these, so near and far
// cover the lattice once.
struct RectUnits {
    int ry0, nrows;  // first row (wrapped) and row count
    int sa, nA, nsegs;  // segments: sa .. sa + nA - 1, then 0 .. (nsegs - nA) - 1
};

__device__ __forceinline__ RectUnits rect_units(const NearRect& r, const GridArgs& g)
{
    RectUnits u;
    if (g.periodic_y) {
        u.nrows = min(r.y1 - r.y0 + 1, g.ny);
        u.ry0 = ((r.y0 % g.ny) + g.ny) % g.ny;
    } else {
        u.ry0 = max(0, r.y0);
        u.nrows = max(0, min(g.ny - 1, r.y1) - u.ry0 + 1);
    }
    const int w = r.x1 - r.x0 + 1;
    if (w >= g.nx) {
        u.sa = 0;
        u.nA = g.nseg;
        u.nsegs = g.nseg;
    } else {
        const int a = ((r.x0 % g.nx) + g.nx) % g.nx;
        const int b = a + w - 1;
        u.sa = a / kSegW;
        if (b < g.nx) {
            u.nA = b / kSegW - u.sa + 1;
            u.nsegs = u.nA;
        } else {
            u.nA = g.nseg - u.sa;
            u.nsegs = u.nA + (b - g.nx) / kSegW + 1;
        }
    }
    return u;
}

// Grid arguments of one lattice of the lattice table.
__device__ __forceinline__ GridArgs lattice_args(const InstDev& I)
{
    GridArgs g;
    g.nx = I.nx;
    g.ny = I.ny;
    g.nxp = I.nxp;
    g.nseg = I.nseg;
    g.periodic_y = I.periodic_y;
    g.periodic_x = I.periodic_x;
    g.omega = I.omega;
    g.gx = I.gx;
    g.u_bot = I.u_bot;
    g.u_top = I.u_top;
    g.u_in = I.u_in;
    g.rho_out = I.rho_out;
    g.uref_c = I.uref_c;
    return g;
}

// Far part: every (row, segment) outside all near regions, i.e. whose entry
// in this step's near map does not carry this step's stamp.  The IB force is
// zero there (its supports lie inside the near regions): an active force flag
// found here means the near regions were too small, ST_NEAR.  The unit runs
// the very code of the single pass (grid_cell), so that the compiler forms
// the same arithmetic and the split repeats the single pass bit for bit.
//
// With `ready`, the pass runs on its own stream without a queue-level wait for
// the IB launch of its step: each block first waits until the IB blocks'
// counter reaches `target` (the count after this step's launch; the counter
// only grows, so any value at or above it is conclusive).  That launch stamped
// this step's near map and ran after the near pass of the previous step on the
// other stream, so both are complete and visible once the count is reached.
// The wait is bounded: a block that gives up raises ST_SYNC and goes on.
__device__ __forceinline__ void wait_for_count(const unsigned long long* ready,
                                               unsigned long long target, int* status)
{
    if (threadIdx.x == 0 && *ready < target) {
        int spins = 0;
        while (__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            // give up after the limit, or at once once another block has
            if (++spins > kSyncSpinLimit ||
                ((spins & 63) == 0 &&
                 (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_SYNC))) {
                atomicOr(status, ST_SYNC);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kSegW * 4) void k_grid_far(
    const T* __restrict__ src, T* __restrict__ dst, const long long* __restrict__ fib_now,
    const int* __restrict__ flags_now, long long* __restrict__ fib_old,
    int* __restrict__ flags_old, const int* __restrict__ near_map, int stamp, int* status,
    GridArgs g, const unsigned long long* ready, unsigned long long target)
{
    // (Row-padding segments run through like the others: letting their blocks
    // leave at once measured slower here, 211.4 -> 212.9 us per fused 4096^2
    // step, the IB launch beside the pass 80 -> 140 us; in the single pass and
    // the batched pass they leave at once.)
    if (ready) wait_for_count(ready, target, status);
    const int b = blockIdx.x;
    const int j = b / kNumXcd;
    const int group = j / g.nseg;
    const int band = group * kNumXcd + (b - j * kNumXcd);
    const int seg = j - group * g.nseg;
    const int lane = threadIdx.x & (kSegW - 1);
    const int y = band * 4 + (threadIdx.x >> 6);
    if (y >= g.ny) return;
    grid_cell<false, true, true>(src, dst, fib_now, flags_now, fib_old, flags_old, g, y, seg, lane,
                                 near_map, stamp, status);
}

// Near part: the (row, segment) units of every capsule's near region, with
// the IB force; `per_cap` blocks of 4 waves share one capsule's units, on the
// capsule's lattice.  Units in several regions are computed more than once,
// with identical results.
template <typename T>
__global__ __launch_bounds__(kSegW * 4) void k_grid_near(
    const T* __restrict__ src, T* __restrict__ dst, const long long* __restrict__ fib_now,
    const int* __restrict__ flags_now, long long* __restrict__ fib_old,
    int* __restrict__ flags_old, const NearRect* __restrict__ rects,
    const CapsuleDev* __restrict__ caps, const InstDev* __restrict__ inst, int per_cap)
{
    const int c = blockIdx.x / per_cap, kb = blockIdx.x - c * per_cap;
    const InstDev& I = inst[caps[c].inst];
    const GridArgs g = lattice_args(I);
    const RectUnits u = rect_units(rects[c], g);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kSegW - 1);
    const int units = u.nrows * u.nsegs;
    for (int q = kb * 4 + wave; q < units; q += per_cap * 4) {
        const int ri = q / u.nsegs, si = q - ri * u.nsegs;
        int y = u.ry0 + ri;
        if (y >= g.ny) y -= g.ny;
        const int seg = si < u.nA ? u.sa + si : si - u.nA;
        grid_cell<false>(src + I.pop_off, dst + I.pop_off, fib_now + I.fib_off,
                         flags_now + I.flag_off, fib_old + I.fib_off, flags_old + I.flag_off, g, y,
                         seg, lane);
    }
}

// Block = 4 wavefronts; a block covers one 64-cell column of a band of
// 4 * ROWS rows, each thread ROWS nodes 4 rows apart (more loads in flight per
// thread).  Workgroups are dealt to the 8 XCDs round-robin; block b is
// remapped so that XCD b % 8 takes whole bands (band = 8 k + b % 8) and walks
// each band along x.  The 8 XCDs then sweep neighbouring bands together
// (accesses spread over all HBM channels), and the cache lines that the
// x-shifted pulls share between neighbouring segments of a band stay in the L2
// of the XCD that owns the band.
template <typename T, int ROWS, bool OPEN, bool NT>
__global__ __launch_bounds__(kSegW * 4) void k_grid_step(
    const T* __restrict__ src, T* __restrict__ dst, const long long* __restrict__ fib_now,
    const int* __restrict__ flags_now, long long* __restrict__ fib_old,
    int* __restrict__ flags_old, GridArgs g)
{
    const int b = blockIdx.x;
    const int j = b / kNumXcd;  // j-th block dealt to this XCD
    const int group = j / g.nseg;
    const int band = group * kNumXcd + (b - j * kNumXcd);
    const int seg = j - group * g.nseg;
    // a row-padding segment (whole block) holds no nodes: 2048 x 512 channel
    // with 32 capsules 38.4 -> 36.8 us per step
    if (seg * kSegW >= g.nx) return;
    const int lane = threadIdx.x & (kSegW - 1);
    const int y0 = band * (4 * ROWS) + (threadIdx.x >> 6);
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
        const int y = y0 + 4 * r;
        if (y < g.ny)
            grid_cell<OPEN, NT>(src, dst, fib_now, flags_now, fib_old, flags_old, g, y, seg, lane);
    }
}

int grid_blocks(int ny, int nseg)
{
    constexpr int R = kGridRowsPerThread;
    const int bands = (ny + 4 * R - 1) / (4 * R);
    const int groups = (bands + kNumXcd - 1) / kNumXcd;
    return groups * nseg * kNumXcd;
}

template <typename T>
hipError_t launch_grid_step(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                            long long* fib_old, int* flags_old, const GridArgs& g, hipStream_t s)
{
    constexpr int R = kGridRowsPerThread;
    const int blocks = grid_blocks(g.ny, g.nseg);
    // streaming stores once the two population buffers outgrow the cache
    const bool nt = 2.0 * 9.0 * g.ny * g.nxp * sizeof(T) > kPlainStoreMaxBytes;
    const dim3 grid((unsigned)blocks), block(kSegW * 4);
    if (g.periodic_x && nt)
        hipLaunchKernelGGL((k_grid_step<T, R, false, true>), grid, block, 0, s, src, dst, fib_now,
                           flags_now, fib_old, flags_old, g);
    else if (g.periodic_x)
        hipLaunchKernelGGL((k_grid_step<T, R, false, false>), grid, block, 0, s, src, dst, fib_now,
                           flags_now, fib_old, flags_old, g);
    else if (nt)
        hipLaunchKernelGGL((k_grid_step<T, R, true, true>), grid, block, 0, s, src, dst, fib_now,
                           flags_now, fib_old, flags_old, g);
    else
        hipLaunchKernelGGL((k_grid_step<T, R, true, false>), grid, block, 0, s, src, dst, fib_now,
                           flags_now, fib_old, flags_old, g);
    return hipGetLastError();
}

// `done`, if given, is marked complete with the kernel itself (the launch's
// stop event), in place of a marker packet recorded behind it on the stream.
template <typename T>
hipError_t launch_grid_far(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                           long long* fib_old, int* flags_old, const int* near_map, int stamp,
                           int* status, const GridArgs& g, hipStream_t s, hipEvent_t done,
                           const unsigned long long* ready, unsigned long long ready_target)
{
    static_assert(kGridRowsPerThread == 1, "k_grid_far takes one row per thread");
    const int blocks = grid_blocks(g.ny, g.nseg);
    if (!done) {
        hipLaunchKernelGGL(k_grid_far<T>, dim3((unsigned)blocks), dim3(kSegW * 4), 0, s, src, dst,
                           fib_now, flags_now, fib_old, flags_old, near_map, stamp, status, g,
                           ready, ready_target);
        return hipGetLastError();
    }
    GridArgs ga = g;
    void* args[] = {&src, &dst, &fib_now, &flags_now, &fib_old, &flags_old, &near_map, &stamp,
                    &status, &ga, &ready, &ready_target};
    return hipExtLaunchKernel(reinterpret_cast<const void*>(&k_grid_far<T>),
                              dim3((unsigned)blocks), dim3(kSegW * 4), args, 0, s, nullptr, done,
                              0);
}

template <typename T>
hipError_t launch_grid_near(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                            long long* fib_old, int* flags_old, const NearRect* rects,
                            const CapsuleDev* caps, const InstDev* inst, int ncap, hipStream_t s)
{
    constexpr int per_cap = 16;
    if (ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_near<T>, dim3((unsigned)(ncap * per_cap)), dim3(kSegW * 4), 0, s,
                       src, dst, fib_now, flags_now, fib_old, flags_old, rects, caps, inst,
                       per_cap);
    return hipGetLastError();
}

// Ensemble of lattices in one launch.  The tiles (a 64-cell segment of a band
// of 4 * ROWS rows) of every lattice form a run that starts at a multiple of
// kNumXcd.  rounds[t / 8] = (lattice, first round of that lattice); tile t is
// processed by a block on XCD t % 8.  Tile orders (ORD):
//   0 banded: the lattice's bands go in groups of 8, which keeps the
//     band-to-XCD mapping above (bands padded to a multiple of 8);
//   1 linear: tile t covers band t / nseg, segment t % nseg of its lattice,
//     the run padded only to a multiple of 8 tiles;
//   2 chunked: the lattice's T tiles in linear order are cut into 8 runs of
//     K = ceil(T / 8) consecutive tiles, one per XCD (tile t covers linear
//     tile (t % 8) K + t / 8), so that most of a tile's x- and y-neighbours sit
//     in the same XCD's L2; same padding as linear.
// With gridDim.x < tiles (a multiple of 8) the launch is persistent: each
// block walks the tiles t = blockIdx.x + k * gridDim.x.
template <typename T, int ROWS, bool OPEN, int ORD, bool FAR>
__global__ __launch_bounds__(kSegW * 4) void k_grid_step_batch(
    const T* __restrict__ src, T* __restrict__ dst, const long long* __restrict__ fib_now,
    const int* __restrict__ flags_now, long long* __restrict__ fib_old,
    int* __restrict__ flags_old, const InstDev* __restrict__ inst,
    const int2* __restrict__ rounds, int tiles, const int* __restrict__ near_map, int stamp,
    int* status)
{
    for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int2 ri = rounds[b / kNumXcd];
        const InstDev& I = inst[ri.x];
        const GridArgs g = lattice_args(I);
        const int lb = b - ri.y * kNumXcd;
        int band, seg;
        if (ORD == 1) {
            band = lb / g.nseg;
            seg = lb - band * g.nseg;
        } else if (ORD == 2) {
            const int bands = (g.ny + 4 * ROWS - 1) / (4 * ROWS);
            const int K = (bands * g.nseg + kNumXcd - 1) / kNumXcd;
            const int t = (lb % kNumXcd) * K + lb / kNumXcd;  // padding tiles land beyond the last band
            band = t / g.nseg;
            seg = t - band * g.nseg;
        } else {
            const int j = lb / kNumXcd;
            const int group = j / g.nseg;
            band = group * kNumXcd + (lb - j * kNumXcd);
            seg = j - group * g.nseg;
        }
        if (seg * kSegW >= g.nx) continue;  // a row-padding segment: no nodes
        const int lane = threadIdx.x & (kSegW - 1);
        const int y0 = band * (4 * ROWS) + (threadIdx.x >> 6);
#pragma unroll
        for (int r = 0; r < ROWS; r++) {
            const int y = y0 + 4 * r;
            if (y >= g.ny) continue;
            // FAR: the far part of the split step, as k_grid_far on one lattice
            grid_cell<OPEN, true, FAR>(src + I.pop_off, dst + I.pop_off, fib_now + I.fib_off,
                                       flags_now + I.flag_off, fib_old + I.fib_off,
                                       flags_old + I.flag_off, g, y, seg, lane,
                                       FAR ? near_map + I.flag_off : nullptr, stamp, status);
        }
    }
}

int grid_blocks_rows(int ny, int nseg, int rows)
{
    const int bands = (ny + 4 * rows - 1) / (4 * rows);
    const int groups = (bands + kNumXcd - 1) / kNumXcd;
    return groups * nseg * kNumXcd;
}

int grid_tiles_linear(int ny, int nseg, int rows)
{
    const int bands = (ny + 4 * rows - 1) / (4 * rows);
    return (bands * nseg + kNumXcd - 1) / kNumXcd * kNumXcd;
}

template <typename T, int R, int ORD>
static void launch_batch_rows(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                              long long* fib_old, int* flags_old, const InstDev* inst,
                              const int2* rounds, int tiles, int grid, bool any_open,
                              const int* near_map, int stamp, int* status, hipStream_t s)
{
    const dim3 gd((unsigned)grid), bd(kSegW * 4);
    if (near_map)  // far part of the split step (periodic lattices only)
        hipLaunchKernelGGL((k_grid_step_batch<T, R, false, ORD, true>), gd, bd, 0, s, src, dst,
                           fib_now, flags_now, fib_old, flags_old, inst, rounds, tiles, near_map,
                           stamp, status);
    else if (any_open)
        hipLaunchKernelGGL((k_grid_step_batch<T, R, true, ORD, false>), gd, bd, 0, s, src, dst,
                           fib_now, flags_now, fib_old, flags_old, inst, rounds, tiles, near_map,
                           stamp, status);
    else
        hipLaunchKernelGGL((k_grid_step_batch<T, R, false, ORD, false>), gd, bd, 0, s, src, dst,
                           fib_now, flags_now, fib_old, flags_old, inst, rounds, tiles, near_map,
                           stamp, status);
}

template <typename T, int ORD>
static hipError_t launch_batch_order(const T* src, T* dst, const long long* fib_now,
                                   const int* flags_now, long long* fib_old, int* flags_old,
                                   const InstDev* inst, const int2* rounds, int tiles, int rows,
                                   int grid, bool any_open, const int* near_map, int stamp,
                                   int* status, hipStream_t s)
{
    if (rows == 1)
        launch_batch_rows<T, 1, ORD>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                     rounds, tiles, grid, any_open, near_map, stamp, status, s);
    else if (rows == 2)
        launch_batch_rows<T, 2, ORD>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                     rounds, tiles, grid, any_open, near_map, stamp, status, s);
    else if (rows == 4)
        launch_batch_rows<T, 4, ORD>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                     rounds, tiles, grid, any_open, near_map, stamp, status, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grid_step_batch(const T* src, T* dst, const long long* fib_now,
                                  const int* flags_now, long long* fib_old, int* flags_old,
                                  const InstDev* inst, const int2* rounds, int tiles, int rows,
                                  int order, int grid, bool any_open, const int* near_map,
                                  int stamp, int* status, hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    if (grid <= 0 || grid > tiles || grid % kNumXcd != 0) return hipErrorInvalidValue;
    if (near_map && any_open) return hipErrorInvalidValue;
    switch (order) {
    case 0:
        return launch_batch_order<T, 0>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                        rounds, tiles, rows, grid, any_open, near_map, stamp,
                                        status, s);
    case 1:
        return launch_batch_order<T, 1>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                        rounds, tiles, rows, grid, any_open, near_map, stamp,
                                        status, s);
    case 2:
        return launch_batch_order<T, 2>(src, dst, fib_now, flags_now, fib_old, flags_old, inst,
                                        rounds, tiles, rows, grid, any_open, near_map, stamp,
                                        status, s);
    default:
        return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ init kernel
// First-order part (3 w_i) e_ix u_ref(y) of the storage reference of slot i in
// row y, in FP64.
template <typename T>
__device__ __forceinline__ double ref_first(const GridArgs& g, int i, int y)
{
    if (g.uref_c == 0.0 || kEx[i] == 0) return 0.0;
    const double w3 = i < 5 ? (double)FirstOrderW<T>::axis : (double)FirstOrderW<T>::diag;
    return w3 * kEx[i] * (g.uref_c * (double)(y * (g.ny - 1 - y)));
}

// Post-collision field whose pull gives f^0 = f^eq(1, u_init(y)) (Eq. 2) at
// every node: slot i at source (x, y) holds the equilibrium at (x, y + e_iy).
template <typename T>
__global__ void k_init(T* pops, GridArgs g, int profile, double ux0, double uy0, double nu)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nxp || y >= g.ny) return;
    const size_t plane = (size_t)g.ny * g.nxp;
    const double H = g.ny - 1;
    for (int i = 0; i < 9; i++) {
        int yd = y + kEy[i];
        if (g.periodic_y) yd = (yd + g.ny) % g.ny;
        else yd = yd < 0 ? 0 : (yd > g.ny - 1 ? g.ny - 1 : yd);
        double ux = 0, uy = 0;
        if (profile == 1) ux = g.u_bot + (g.u_top - g.u_bot) * yd / H;
        else if (profile == 2) ux = g.gx / (2.0 * nu) * yd * (H - yd);
        else if (profile == 3) { ux = ux0; uy = uy0; }
        else if (profile == 4) ux = 4.0 * g.u_in * yd * (H - yd) / (H * H);
        const double eu = kEx[i] * ux + kEy[i] * uy;
        const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double dev = w * (3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
        pops[i * plane + (size_t)y * g.nxp + x] = x < g.nx ? (T)(dev - ref_first<T>(g, i, y)) : T(0);
    }
}

template <typename T>
hipError_t launch_init(T* pops, const GridArgs& g, int profile, double ux0, double uy0, double nu,
                       hipStream_t s)
{
    dim3 block(256), grid((g.nxp + 255) / 256, g.ny);
    hipLaunchKernelGGL(k_init<T>, grid, block, 0, s, pops, g, profile, ux0, uy0, nu);
    return hipGetLastError();
}

// --------------------------------------------------------------- IB kernel

template <typename T>
__device__ __forceinline__ void two_sum(T a, T b, T& s, T& e)
{
#pragma clang fp contract(off)
    s = a + b;
    const T bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Adds d to the compensated coordinate (hi, lo).
template <typename T>
__device__ __forceinline__ void comp_add(T& hi, T& lo, T d)
{
#pragma clang fp contract(off)
    T s, e;
    two_sum(hi, d, s, e);
    e += lo;
    T s2, e2;
    two_sum(s, e, s2, e2);
    hi = s2;
    lo = e2;
}

// MLS shape functions of Eq. 9 at p = (px, py), given relative to an integer
// origin.  Support: the 3x3 nodes around floor(p + 1/2).  Weight
// exp(-(|x_k - p| / (r_w alpha))^2) with r_w = 2.6, alpha = 0.3.  Linear basis
// centred on p.  The 3x3 moment matrix is accumulated and inverted (cofactors)
// in FP64.  Outputs: centre (cx, cy), phi (value) and, if G, the slope rows
// (dphi/dx, dphi/dy) of the local fit.
template <typename T, bool G>
__device__ __forceinline__ void mls(T px, T py, int& cx, int& cy, T* phi, T* gx, T* gy)
{
    cx = (int)floor(px + T(0.5));
    cy = (int)floor(py + T(0.5));
    const T inv2 = T(1.0 / (2.6 * 0.3 * 2.6 * 0.3));
    T w[9], rx[9], ry[9];
    double a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        rx[k] = (T)(cx + k % 3 - 1) - px;
        ry[k] = (T)(cy + k / 3 - 1) - py;
        w[k] = exp(-(rx[k] * rx[k] + ry[k] * ry[k]) * inv2);
        const double W = w[k], X = rx[k], Y = ry[k];
        a00 += W;
        a01 += W * X;
        a02 += W * Y;
        a11 += W * X * X;
        a12 += W * X * Y;
        a22 += W * Y * Y;
    }
    const double c00 = a11 * a22 - a12 * a12;
    const double c01 = a02 * a12 - a01 * a22;
    const double c02 = a01 * a12 - a02 * a11;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    const double id = 1.0 / det;
    const double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    double i11 = 0, i12 = 0, i22 = 0;
    if (G) {
        i11 = (a00 * a22 - a02 * a02) * id;
        i12 = (a01 * a02 - a00 * a12) * id;
        i22 = (a00 * a11 - a01 * a01) * id;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const double W = w[k], X = rx[k], Y = ry[k];
        phi[k] = (T)(W * (i00 + i01 * X + i02 * Y));
        if (G) {
            gx[k] = (T)(W * (i01 + i11 * X + i12 * Y));
            gy[k] = (T)(W * (i02 + i12 * X + i22 * Y));
        }
    }
}

// Eq. 8 interpolation of the velocity at p.
template <typename T>
__device__ __forceinline__ void interp_u(const Patch<T>& P, T px, T py, T& Ux, T& Uy, int& st)
{
    int cx, cy;
    T phi[9];
    mls<T, false>(px, py, cx, cy, phi, nullptr, nullptr);
    Ux = Uy = T(0);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        int idx;
        if (!patch_index(P, cx, cy, k, idx)) { st |= ST_PATCH; continue; }
        if (isnan(P.drho[idx])) { st |= ST_WALL; continue; }
        Ux += phi[k] * P.ux[idx];
        Uy += phi[k] * P.uy[idx];
    }
}

// Probe state for Eqs. 15-16: pressure deviation c_s^2 (rho - 1) and the
// velocity gradient G[a][b] = d u_a / d x_b from the slope rows of the fit.
template <typename T>
__device__ __forceinline__ void probe(const Patch<T>& P, T px, T py, T& dp, T (&Gr)[2][2], int& st)
{
    int cx, cy;
    T phi[9], gx[9], gy[9];
    mls<T, true>(px, py, cx, cy, phi, gx, gy);
    T r = 0, g00 = 0, g01 = 0, g10 = 0, g11 = 0;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        int idx;
        if (!patch_index(P, cx, cy, k, idx)) { st |= ST_PATCH; continue; }
        const T d = P.drho[idx];
        if (isnan(d)) { st |= ST_WALL; continue; }
        const T u = P.ux[idx], v = P.uy[idx];
        r += phi[k] * d;
        g00 += gx[k] * u;
        g01 += gy[k] * u;
        g10 += gx[k] * v;
        g11 += gy[k] * v;
    }
    dp = r * T(1.0 / 3.0);
    Gr[0][0] = g00;
    Gr[0][1] = g01;
    Gr[1][0] = g10;
    Gr[1][1] = g11;
}

// Scratch arrays of the IB kernel, each max_nv long.
template <typename T>
struct Scratch {
    T* px;  // node positions (high parts, relative to the reference point)
    T* py;
    T* qx;  // low parts of the compensated positions
    T* qy;
    T* dx;  // last displacement d^n
    T* dy;
    T* ux;  // node velocity u_v^n
    T* uy;
    T* l0;  // stress-free length (high, low), stretching constant, turning angle
    T* l0l;
    T* ks;
    T* th0;
    T* t[kNodeScratch];
};

// Edge vector x_m - x_l from compensated coordinates: the difference of the
// high parts of nearby nodes is exact, the low parts restore the rest.
template <typename T>
__device__ __forceinline__ void edge(const Scratch<T>& S, int l, int m, T& tx, T& ty)
{
    tx = (S.px[m] - S.px[l]) + (S.qx[m] - S.qx[l]);
    ty = (S.py[m] - S.py[l]) + (S.qy[m] - S.qy[l]);
}

// Error-free product a * b = p + e (FMA).
template <typename T>
__device__ __forceinline__ void two_prod(T a, T b, T& p, T& e)
{
#pragma clang fp contract(off)
    p = a * b;
    e = fma(a, b, -p);
}

// Stretch of element l -> m, len - l0, and len.  In FP32 the two lengths are
// nearly equal, so the difference is formed as (len^2 - l0^2) / (len + l0)
// with len^2 and l0^2 carried as unevaluated float pairs: the edge vector from
// the compensated coordinates, l0 from its stored high and low parts.
template <typename T>
__device__ __forceinline__ T stretch(const Scratch<T>& S, int l, int m, T l0h, T l0l, T& len)
{
#pragma clang fp contract(off)
    T hx, ex, hy, ey;
    two_sum(S.px[m], -S.px[l], hx, ex);
    two_sum(S.py[m], -S.py[l], hy, ey);
    const T lx = ex + (S.qx[m] - S.qx[l]);
    const T ly = ey + (S.qy[m] - S.qy[l]);
    T p1, e1, p2, e2, s, es, q, eq;
    two_prod(hx, hx, p1, e1);
    two_prod(hy, hy, p2, e2);
    two_sum(p1, p2, s, es);
    const T lo = es + e1 + e2 + T(2) * (hx * lx + hy * ly) + (lx * lx + ly * ly);
    two_prod(l0h, l0h, q, eq);
    const T lo0 = eq + T(2) * l0h * l0l + l0l * l0l;
    const T diff = (s - q) + (lo - lo0);
    len = sqrt(s + lo);
    return diff / (len + (l0h + l0l));
}

// Eqs. 10-14, per element l -> l+1 (the stretching and area terms) and per node
// v (the bending terms); the caller sums them onto the nodes with
// membrane_node_force.  Stretch: k_s (len - l0) t / len on node l and its
// negative on node l+1.  Area: F_l = -k_a (1 - A/A0) c_s^2 n- len, half to each
// end, with A the FP64 enclosed area.  Bending (outer terms of Eq. 13 as
// printed, the middle node takes minus their sum): k_b sin(theta - theta0) n /
// len on the two neighbours.  Results in S.t[14..21].
template <typename T>
__device__ __forceinline__ void membrane_terms(const Scratch<T>& S, int l, int nv, double kb, T cA,
                                               float max_edge, int& st)
{
    const int m = l + 1 == nv ? 0 : l + 1;
    T tx, ty, len;
    edge(S, l, m, tx, ty);
    const T c = S.ks[l] * stretch(S, l, m, S.l0[l], S.l0l[l], len) / len;
    // an element longer than the set limit (the forcing may leave holes, Sec. 3.2)
    if (max_edge > 0.0f && !(len <= (T)max_edge)) st |= ST_EDGE;
    const T ax = cA * ty, ay = -cA * tx;
    S.t[14][l] = c * tx + ax;  // onto node l
    S.t[15][l] = c * ty + ay;
    S.t[16][l] = -c * tx + ax;  // onto node l+1
    S.t[17][l] = -c * ty + ay;
    if (kb != 0.0) {
        const int v = l, vl = v == 0 ? nv - 1 : v - 1, vr = m;
        T ax2, ay2, bx, by;
        edge(S, vl, v, ax2, ay2);
        edge(S, v, vr, bx, by);
        const T la = sqrt(ax2 * ax2 + ay2 * ay2), lb = sqrt(bx * bx + by * by);
        const T th = atan2(ax2 * by - ay2 * bx, ax2 * bx + ay2 * by);
        const T sn = (T)kb * sin(th - S.th0[v]);
        S.t[18][v] = sn * ay2 / (la * la);  // k_b s n_left / l_left, n_left = (a_y, -a_x)/l
        S.t[19][v] = -sn * ax2 / (la * la);
        S.t[20][v] = sn * by / (lb * lb);
        S.t[21][v] = -sn * bx / (lb * lb);
    }
}

// The FP64 enclosed area (Green's theorem over the compensated positions) as
// this thread's share of the sum; block_sum / the wave partials complete it.
template <typename T>
__device__ __forceinline__ double area_share(const Scratch<T>& S, int nv)
{
    double acc = 0.0;
    for (int l = threadIdx.x; l < nv; l += blockDim.x) {
        const int m = l + 1 == nv ? 0 : l + 1;
        const double xl = (double)S.px[l] + (double)S.qx[l], yl = (double)S.py[l] + (double)S.qy[l];
        const double xm = (double)S.px[m] + (double)S.qx[m], ym = (double)S.py[m] + (double)S.qy[m];
        acc += xl * ym - xm * yl;
    }
    return acc;
}

// Half element area force per (t_y, -t_x), and the area-drift flag.
__device__ __forceinline__ double area_coefficient(double A, double A0, double ka, float max_dA,
                                                   int& st)
{
    if (max_dA > 0.0f && threadIdx.x == 0 && !(fabs(A / A0 - 1.0) <= (double)max_dA)) st |= ST_AREA;
    return 0.5 * ka * (1.0 - A / A0) / 3.0;
}

// Dynamic step 7 force terms in one pass.  Given the positions and the staged
// patch, the membrane forces (Eqs. 10-14), the probes of Eqs. 15-16 and the
// tentative velocity of Eq. 23 are independent of one another, so they are
// evaluated side by side, each kind on its own waves: the membrane terms
// (membrane_terms), per (element, side) a probe (S.t[0..7]: pressure deviation
// and the symmetric velocity-gradient terms), per node the interpolated fluid
// velocity (S.t[12], S.t[13]).  A second pass combines each element's two
// probes into its half force (S.t[10], S.t[11]); the node update adds the
// nodal sums itself (dynamic_node_forces).  Two block barriers in all (one
// after the other these passes took seven).  A: the FP64 enclosed area,
// reduced by the caller from the same positions.
template <typename T>
__device__ void dynamic_forces(const Scratch<T>& S, const Patch<T>& P, int nv, double kb,
                               double ka, double A0, double A, T nu, float max_edge,
                               float max_dA, int& st)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const T cA = (T)area_coefficient(A, A0, ka, max_dA, st);
    const size_t stride = S.t[1] - S.t[0];
    // item ranges start on wave boundaries, so that no wave mixes two kinds;
    // three loops rather than one with three branches keep the register
    // pressure of each kind to itself
    const int n1 = (nv + 63) & ~63, n2 = n1 + ((2 * nv + 63) & ~63);
    for (int l = tid; l < nv; l += nt) membrane_terms(S, l, nv, kb, cA, max_edge, st);
    for (int w = tid - n1; w < 2 * nv; w += nt) {
        if (w < 0) continue;
        const int l = w >> 1, side = w & 1;
        const int m = l + 1 == nv ? 0 : l + 1;
        T tx, ty;
        edge(S, l, m, tx, ty);
        const T len = sqrt(tx * tx + ty * ty);
        const T sg = side ? T(-1.2) : T(1.2);
        const T nx = ty / len, ny = -tx / len;  // outward normal n+
        const T xc = T(0.5) * (S.px[l] + S.px[m]), yc = T(0.5) * (S.py[l] + S.py[m]);
        T dp, G[2][2];
        probe(P, xc + sg * nx, yc + sg * ny, dp, G, st);
        T* o = S.t[0] + (size_t)side * 4 * stride;
        o[l] = dp;
        o[stride + l] = T(2) * G[0][0];
        o[2 * stride + l] = T(2) * G[1][1];
        o[3 * stride + l] = G[0][1] + G[1][0];
    }
    for (int v = tid - n2; v < nv; v += nt) {
        if (v < 0) continue;
        interp_u(P, S.px[v], S.py[v], S.t[12][v], S.t[13][v], st);
    }
    __syncthreads();
    // each element's hydrodynamic force (tau+ - tau-) . n+ len, tau = nu (G + G^T),
    // half to each end node
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        T tx, ty;
        edge(S, l, m, tx, ty);
        const T len = sqrt(tx * tx + ty * ty);
        const T nx = ty / len, ny = -tx / len;
        const T dpr = S.t[0][l] - S.t[4][l];
        const T d00 = S.t[1][l] - S.t[5][l];
        const T d11 = S.t[2][l] - S.t[6][l];
        const T d01 = S.t[3][l] - S.t[7][l];
        const T fx = (-dpr * nx + nu * (d00 * nx + d01 * ny)) * len;
        const T fy = (-dpr * ny + nu * (d01 * nx + d11 * ny)) * len;
        S.t[10][l] = T(0.5) * fx;
        S.t[11][l] = T(0.5) * fy;
    }
    __syncthreads();
}

// Nodal sum of the membrane terms (S.t[14..21]) for node v.
template <typename T>
__device__ __forceinline__ void membrane_node_force(const Scratch<T>& S, int v, int nv, double kb,
                                                    T& fix, T& fiy)
{
    const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
    const T *Px = S.t[14], *Py = S.t[15], *Qx = S.t[16], *Qy = S.t[17];
    const T *BLx = S.t[18], *BLy = S.t[19], *BRx = S.t[20], *BRy = S.t[21];
    fix = Px[v] + Qx[vl];
    fiy = Py[v] + Qy[vl];
    if (kb != 0.0) {
        fix += BRx[vl] + BLx[vr] - BLx[v] - BRx[v];
        fiy += BRy[vl] + BLy[vr] - BLy[v] - BRy[v];
    }
}

// Nodal sums of the Dynamic force pass for node v: membrane (fix, fiy) and
// hydrodynamic (fex, fey, the halves of its two elements).  The node update
// takes them directly, which spares a pass and its barrier.
template <typename T>
__device__ __forceinline__ void dynamic_node_forces(const Scratch<T>& S, int v, int nv, double kb,
                                                    T& fix, T& fiy, T& fex, T& fey)
{
    membrane_node_force(S, v, nv, kb, fix, fiy);
    const int vl = v == 0 ? nv - 1 : v - 1;
    fex = S.t[10][v] + S.t[10][vl];
    fey = S.t[11][v] + S.t[11][vl];
}

// Kinematic step i and the spreading weights of step iii in one pass: after
// the FP64 area reduction, the membrane terms (membrane_terms) and, on their
// own waves, each node's MLS fit at x^n (cache_weights) are independent, so
// they run side by side; the caller then adds the nodal sums
// (membrane_node_force).
template <typename T>
__device__ void kinematic_forces(const Scratch<T>& S, int nv, double kb, double ka, double A0,
                                 double (*red)[8], float max_edge, float max_dA, int& st)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double acc[1] = {area_share(S, nv)};
    block_sum<1>(acc, red);
    const T cA = (T)area_coefficient(0.5 * acc[0], A0, ka, max_dA, st);
    const int n1 = (nv + 63) & ~63;
    for (int l = tid; l < nv; l += nt) membrane_terms(S, l, nv, kb, cA, max_edge, st);
    for (int v = tid - n1; v < nv; v += nt) {
        if (v < 0) continue;
        int cx, cy;
        T phi[9];
        mls<T, false>(S.px[v], S.py[v], cx, cy, phi, nullptr, nullptr);
        cache_weights(S, v, cx, cy, phi);  // c_v = 1
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ long long to_fix(T v, int& st)
{
    if (!(fabs(v) < (T)kFixLimit)) {
        st |= isnan(v) ? ST_NONFINITE : ST_OVERFLOW;
        return 0;
    }
    return (long long)rint((double)v * kFixScale);
}

// One spreading contribution (Dynamic step 3, Kinematic step iii): the value
// (vx, vy) = c phi_k F goes to support node k of the 3x3 support centred on
// (cx, cy), relative to the reference point.
// (bx, by): the reference point reduced onto periodic axes (wrap_ref).
struct SpreadRef {
    long long rx, ry;
    int bx, by;
};

__device__ __forceinline__ SpreadRef spread_ref(const GridArgs& g, long long refx, long long refy)
{
    SpreadRef r;
    r.rx = refx;
    r.ry = refy;
    r.bx = g.periodic_x ? wrap_ref(refx, g.nx) : 0;
    r.by = g.periodic_y ? wrap_ref(refy, g.ny) : 0;
    return r;
}

template <typename T>
__device__ __forceinline__ void spread_one(const IBArgs<T>& a, const GridArgs& g,
                                           const SpreadRef& r, int cx, int cy, int k, T vx, T vy,
                                           int& st)
{
    int gy, gx;
    if (g.periodic_y) {
        gy = wrap_add(r.by, cy + k / 3 - 1, g.ny);
    } else {
        const long long v = r.ry + cy + k / 3 - 1;
        if (v < 1 || v > g.ny - 2) { st |= ST_WALL; return; }
        gy = (int)v;
    }
    if (g.periodic_x) {
        gx = wrap_add(r.bx, cx + k % 3 - 1, g.nx);
    } else {
        const long long v = r.rx + cx + k % 3 - 1;
        if (v < 1 || v > g.nx - 2) { st |= ST_WALL; return; }
        gx = (int)v;
    }
    const long long fx = to_fix(vx, st), fy = to_fix(vy, st);
    const size_t cell = (size_t)gy * g.nxp + (size_t)gx;
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(a.fib_next + 2 * cell);
    atomicAdd(dst, (unsigned long long)fx);
    atomicAdd(dst + 1, (unsigned long long)fy);
    a.flags_next[gy * g.nseg + gx / kSegW] = 1;
}

// MLS weights of node v cached for the spreading: phi_0..7 in S.t[0..7],
// phi_8 in S.t[12], support centre in S.t[10..11] (exact small integers).
template <typename T>
__device__ __forceinline__ void cache_weights(const Scratch<T>& S, int v, int cx, int cy,
                                              const T* phi)
{
#pragma unroll
    for (int k = 0; k < 8; k++) S.t[k][v] = phi[k];
    S.t[12][v] = phi[8];
    S.t[10][v] = (T)cx;
    S.t[11][v] = (T)cy;
}

// Spreads the cached c_v F_v (S.t[8..9]) with the cached weights; one work
// item per (node, support node).
template <typename T>
__device__ __forceinline__ void spread_cached(const IBArgs<T>& a, const GridArgs& g,
                                              const Scratch<T>& S, int nv, long long refx,
                                              long long refy, int& st)
{
    const T* base = S.t[0];
    const size_t stride = S.t[1] - S.t[0];  // the scratch arrays are contiguous
    const SpreadRef r = spread_ref(g, refx, refy);
    for (int w = threadIdx.x; w < 9 * nv; w += blockDim.x) {
        const int v = w / 9, k = w - 9 * v;
        const T phi = base[(size_t)(k < 8 ? k : 12) * stride + v];
        spread_one(a, g, r, (int)S.t[10][v], (int)S.t[11][v], k, phi * S.t[8][v],
                   phi * S.t[9][v], st);
    }
}

// The same spreading through a pre-sum over the patch box in LDS: each
// (node, support node) contribution is added there as 64-bit fixed point
// (integer sums, so their order does not matter and the force level gets the
// same bits), then every touched cell adds its two sums to the level with one
// pair of global atomics and raises its segment flag.  The sums take the
// patch arrays (dead once the forcing has interpolated); the caller checks
// that 20 bytes per patch cell fit there.  A contribution outside the box
// goes straight to the level.
template <typename T>
__device__ __forceinline__ void spread_patch(const IBArgs<T>& a, const GridArgs& g,
                                             const Scratch<T>& S, const Patch<T>& P, int nv,
                                             long long refx, long long refy, int& st)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ncell = P.W * P.H;
    unsigned long long* sx = reinterpret_cast<unsigned long long*>(P.drho);
    unsigned long long* sy = sx + ncell;
    int* touched = reinterpret_cast<int*>(sy + ncell);
    for (int i = tid; i < ncell; i += nt) {
        sx[i] = 0;
        sy[i] = 0;
        touched[i] = 0;
    }
    __syncthreads();
    const T* base = S.t[0];
    const size_t stride = S.t[1] - S.t[0];  // the scratch arrays are contiguous
    const SpreadRef r = spread_ref(g, refx, refy);
    for (int w = tid; w < 9 * nv; w += nt) {
        const int v = w / 9, k = w - 9 * v;
        const T phi = base[(size_t)(k < 8 ? k : 12) * stride + v];
        const int cx = (int)S.t[10][v], cy = (int)S.t[11][v];
        const T vx = phi * S.t[8][v], vy = phi * S.t[9][v];
        int idx;
        if (!patch_index(P, cx, cy, k, idx)) {
            spread_one(a, g, r, cx, cy, k, vx, vy, st);
            continue;
        }
        if (!g.periodic_y) {  // walls: as spread_one
            const long long yv = r.ry + cy + k / 3 - 1;
            if (yv < 1 || yv > g.ny - 2) { st |= ST_WALL; continue; }
        }
        if (!g.periodic_x) {
            const long long xv = r.rx + cx + k % 3 - 1;
            if (xv < 1 || xv > g.nx - 2) { st |= ST_WALL; continue; }
        }
        const long long fx = to_fix(vx, st), fy = to_fix(vy, st);
        atomicAdd(&sx[idx], (unsigned long long)fx);
        atomicAdd(&sy[idx], (unsigned long long)fy);
        touched[idx] = 1;
    }
    __syncthreads();
    const int bx = g.periodic_x ? wrap_ref(refx + P.ox, g.nx) : 0;
    const int by = g.periodic_y ? wrap_ref(refy + P.oy, g.ny) : 0;
    for (int i = tid; i < ncell; i += nt) {
        if (!touched[i]) continue;
        const int lx = i % P.W, ly = i / P.W;
        const int gx = g.periodic_x ? wrap_add(bx, lx, g.nx) : (int)(refx + P.ox + lx);
        const int gy = g.periodic_y ? wrap_add(by, ly, g.ny) : (int)(refy + P.oy + ly);
        const size_t cell = (size_t)gy * g.nxp + (size_t)gx;
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(a.fib_next + 2 * cell);
        if (sx[i]) atomicAdd(dst, sx[i]);
        if (sy[i]) atomicAdd(dst + 1, sy[i]);
        a.flags_next[gy * g.nseg + gx / kSegW] = 1;
    }
}

// Sec. 3 diagnostics of the polygon (FP64): area, perimeter, centroid, central
// second moments of area -> Taylor deformation of the equivalent ellipse,
// swelling ratio, perimeter and area change.
template <typename T>
__device__ void diagnostics(const IBArgs<T>& a, const CapsuleDev& cap, int c, double (*red)[8])
{
    const int tid = threadIdx.x, nt = blockDim.x, nv = cap.nv, off = cap.node_offset;
    const T* N = a.nodes;
    const size_t S = a.node_stride;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        const double x0 = (double)N[NF_HX * S + off + l] + (double)N[NF_LX * S + off + l];
        const double y0 = (double)N[NF_HY * S + off + l] + (double)N[NF_LY * S + off + l];
        const double x1 = (double)N[NF_HX * S + off + m] + (double)N[NF_LX * S + off + m];
        const double y1 = (double)N[NF_HY * S + off + m] + (double)N[NF_LY * S + off + m];
        const double cr = x0 * y1 - x1 * y0;
        v[0] += cr;
        v[1] += sqrt((x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0));
        v[2] += (x0 + x1) * cr;
        v[3] += (y0 + y1) * cr;
        v[4] += (x0 * x0 + x0 * x1 + x1 * x1) * cr;
        v[5] += (y0 * y0 + y0 * y1 + y1 * y1) * cr;
        v[6] += (x0 * y1 + 2.0 * x0 * y0 + 2.0 * x1 * y1 + x1 * y0) * cr;
    }
    block_sum<7>(v, red);
    if (tid == 0) {
        const double A = 0.5 * v[0], P = v[1];
        const double cx = v[2] / (6.0 * A), cy = v[3] / (6.0 * A);
        const double jxx = v[4] / 12.0 - A * cx * cx;
        const double jyy = v[5] / 12.0 - A * cy * cy;
        const double jxy = v[6] / 24.0 - A * cx * cy;
        const double tr = 0.5 * (jxx + jyy);
        const double disc = sqrt(0.25 * (jxx - jyy) * (jxx - jyy) + jxy * jxy);
        const double l1 = tr + disc, l2 = fmax(tr - disc, 0.0);
        const double sa = sqrt(l1), sb = sqrt(l2);
        double* d = a.diag + (size_t)c * kDiagStride;
        d[0] = A;
        d[1] = P;
        d[2] = cap.ref_x + cx;
        d[3] = cap.ref_y + cy;
        d[4] = (sa - sb) / (sa + sb);
        d[5] = 4.0 * M_PI * A / (P * P);
        d[6] = (P - cap.P0) / cap.P0;
        d[7] = A / cap.A0 - 1.0;
        d[8] = jxx;
        d[9] = jyy;
        d[10] = jxy;
        d[11] = cap.A0;
        d[12] = cap.P0;
    }
}

// Rigid particle start-up (reading, as for membranes): u^0 = u^{-1} = mean of
// the interpolated fluid velocity at the nodes, w^0 = w^{-1} = the
// least-squares rigid rotation of those velocities about the centroid; the
// nodes take the rigid-body velocity, and d^0 = u_v^0.
template <typename T>
__device__ void rigid_prime(const IBArgs<T>& a, const Scratch<T>& S, const Patch<T>& P,
                            CapsuleDev& cap, int c, int& st, double (*red)[8])
{
    const int tid = threadIdx.x, nt = blockDim.x, nv = cap.nv, off = cap.node_offset;
    const size_t NS = a.node_stride;
    T* N = a.nodes;
    const double Xr = cap.rX - cap.ref_x, Yr = cap.rY - cap.ref_y;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int v = tid; v < nv; v += nt) {
        T Ux, Uy;
        interp_u(P, S.px[v], S.py[v], Ux, Uy, st);
        const double rx = (double)S.px[v] + (double)S.qx[v] - Xr;
        const double ry = (double)S.py[v] + (double)S.qy[v] - Yr;
        acc[0] += (double)Ux;
        acc[1] += (double)Uy;
        acc[2] += rx * (double)Uy - ry * (double)Ux;
        acc[3] += rx * rx + ry * ry;
    }
    block_sum<4>(acc, red);
    const double ux = acc[0] / nv, uy = acc[1] / nv, w = acc[2] / acc[3];
    for (int v = tid; v < nv; v += nt) {
        const double rx = (double)S.px[v] + (double)S.qx[v] - Xr;
        const double ry = (double)S.py[v] + (double)S.qy[v] - Yr;
        const T vx = (T)(ux - w * ry), vy = (T)(uy + w * rx);
        N[NF_UX * NS + cap.node_offset + v] = vx;
        N[NF_UY * NS + cap.node_offset + v] = vy;
        N[NF_DX * NS + off + v] = vx;
        N[NF_DY * NS + off + v] = vy;
        S.ux[v] = vx;
        S.uy[v] = vy;
        S.dx[v] = vx;
        S.dy[v] = vy;
    }
    cap.ru[0] = cap.rum1[0] = ux;
    cap.ru[1] = cap.rum1[1] = uy;
    cap.rw = cap.rwm1 = w;
    if (tid == 0) {
        a.caps[c].ru[0] = a.caps[c].rum1[0] = ux;
        a.caps[c].ru[1] = a.caps[c].rum1[1] = uy;
        a.caps[c].rw = a.caps[c].rwm1 = w;
    }
}

// Rigid particle update closing step n-1 (Sec. 2.3.1): force and torque from
// the stresses at the outer probes x_c + 1.2 n+ (Eqs. 17-18; pressure as the
// deviation c_s^2 (rho - 1), torque about the centroid with the element
// centroid as lever point) plus the contact forces on the nodes; velocities by
// Eqs. 19-20 from F/m and M/I; (reading) X += u dt, theta += w dt; the nodes
// go to X + R(theta) r0 with the rigid-body velocity.  New positions are left
// in S.t[4..7] with their sum in csum, for the common re-basing.
template <typename T>
__device__ void rigid_update(const IBArgs<T>& a, const Scratch<T>& S, const Patch<T>& P,
                             CapsuleDev& cap, int c, int& st, double (*red)[8], double (&csum)[2])
{
    const int tid = threadIdx.x, nt = blockDim.x, nv = cap.nv, off = cap.node_offset;
    const size_t NS = a.node_stride;
    T* N = a.nodes;
    const double Xr = cap.rX - cap.ref_x, Yr = cap.rY - cap.ref_y;
    const T nu = (T)cap.nu;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        T tx, ty;
        edge(S, l, m, tx, ty);
        const T len = sqrt(tx * tx + ty * ty);
        const T nx = ty / len, ny = -tx / len;
        const T xc = T(0.5) * (S.px[l] + S.px[m]), yc = T(0.5) * (S.py[l] + S.py[m]);
        T dp, G[2][2];
        probe(P, xc + T(1.2) * nx, yc + T(1.2) * ny, dp, G, st);
        const T t00 = nu * T(2) * G[0][0], t11 = nu * T(2) * G[1][1];
        const T t01 = nu * (G[0][1] + G[1][0]);
        const double fx = (double)((t00 * nx + t01 * ny - dp * nx) * len);
        const double fy = (double)((t01 * nx + t11 * ny - dp * ny) * len);
        acc[0] += fx;
        acc[1] += fy;
        acc[2] += ((double)xc - Xr) * fy - ((double)yc - Yr) * fx;
    }
    if (a.contact) {
        for (int v = tid; v < nv; v += nt) {
            const double fx = (double)N[NF_CX * NS + off + v], fy = (double)N[NF_CY * NS + off + v];
            const double rx = (double)S.px[v] + (double)S.qx[v] - Xr;
            const double ry = (double)S.py[v] + (double)S.qy[v] - Yr;
            acc[0] += fx;
            acc[1] += fy;
            acc[2] += rx * fy - ry * fx;
        }
    }
    block_sum<3>(acc, red);
    const double ux = 2.0 / 3.0 * (2.0 * cap.ru[0] - 0.5 * cap.rum1[0] + acc[0] / cap.rm);
    const double uy = 2.0 / 3.0 * (2.0 * cap.ru[1] - 0.5 * cap.rum1[1] + acc[1] / cap.rm);
    const double w = 2.0 / 3.0 * (2.0 * cap.rw - 0.5 * cap.rwm1 + acc[2] / cap.rI);
    const double Xn = Xr + ux, Yn = Yr + uy, th = cap.rth + w;
    const double cs = cos(th), sn = sin(th);
    for (int v = tid; v < nv; v += nt) {
        const double r0x = (double)N[NF_R0X * NS + off + v], r0y = (double)N[NF_R0Y * NS + off + v];
        const double rx = cs * r0x - sn * r0y, ry = sn * r0x + cs * r0y;
        const double x = Xn + rx, y = Yn + ry;
        const T hx = (T)x, hy = (T)y;
        const T lx = (T)(x - (double)hx), ly = (T)(y - (double)hy);
        const T dx = (T)(x - ((double)S.px[v] + (double)S.qx[v]));
        const T dy = (T)(y - ((double)S.py[v] + (double)S.qy[v]));
        if (!(fabs(dx) < T(1) && fabs(dy) < T(1))) st |= ST_MOVE;
        const T vx = (T)(ux - w * ry), vy = (T)(uy + w * rx);
        N[NF_DX * NS + off + v] = dx;
        N[NF_DY * NS + off + v] = dy;
        N[NF_UX * NS + off + v] = vx;
        N[NF_UY * NS + off + v] = vy;
        S.dx[v] = dx;
        S.dy[v] = dy;
        S.ux[v] = vx;
        S.uy[v] = vy;
        S.t[4][v] = hx;
        S.t[5][v] = hy;
        S.t[6][v] = lx;
        S.t[7][v] = ly;
        csum[0] += (double)hx;
        csum[1] += (double)hy;
    }
    cap.rum1[0] = cap.ru[0];
    cap.rum1[1] = cap.ru[1];
    cap.rwm1 = cap.rw;
    cap.ru[0] = ux;
    cap.ru[1] = uy;
    cap.rw = w;
    cap.rX = cap.ref_x + Xn;
    cap.rY = cap.ref_y + Yn;
    cap.rth = th;
    if (tid == 0) {
        CapsuleDev& o = a.caps[c];
        o.rum1[0] = cap.rum1[0];
        o.rum1[1] = cap.rum1[1];
        o.rwm1 = cap.rwm1;
        o.ru[0] = ux;
        o.ru[1] = uy;
        o.rw = w;
        o.rX = cap.rX;
        o.rY = cap.rY;
        o.rth = th;
        o.rF[0] = acc[0];
        o.rF[1] = acc[1];
        o.rM = acc[2];
    }
}

// One block per capsule.  Phases (bit set):
//   PH_PRIME  start-up of a capsule not yet started: u_v^0 = U(x^0), d^0 = U(x^0)
//   PH_B      node update closing step n-1 from the fields after its collision:
//             Dynamic steps 7-8 (Eqs. 21-24), Kinematic steps vii-viii (Eq. 25)
//   PH_A      forcing of step n: Dynamic steps 1-3 (direct forcing, spreading
//             with c_v = node arc length), Kinematic steps i-iii (internal
//             forces, c_v = 1)
//   PH_DIAG   diagnostics of the current shape only
template <typename T, bool DYN>
__device__ __forceinline__ void ib_block(const IBArgs<T>& a0, unsigned char* smem,
                                         double (*red)[8])
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int c = blockIdx.x;
    // the patch box of the last launch (used below) is loaded beside the record
    const int4 hint0 = a0.hints ? a0.hints[c] : make_int4(0, 0, 0, 0);
    CapsuleDev cap = a0.caps[c];
    // the capsule's lattice: buffer offsets and sizes
    IBArgs<T> a = a0;
    a.pops += cap.pop_off;
    a.fib_prev += cap.fib_off;
    a.fib_next += cap.fib_off;
    a.flags_next += cap.flag_off;
    if (a.near_map) a.near_map += cap.flag_off;
    GridArgs g;
    g.nx = cap.nx;
    g.ny = cap.ny;
    g.nxp = cap.nxp;
    g.nseg = cap.nseg;
    g.periodic_y = cap.periodic_y;
    g.periodic_x = cap.periodic_x;
    g.omega = 0.0;
    g.gx = cap.gx;
    g.u_bot = g.u_top = 0.0;  // wall rows and open-channel columns are never staged
    g.u_in = 0.0;
    g.rho_out = 1.0;
    g.uref_c = cap.uref_c;
    const int nv = cap.nv, off = cap.node_offset;
    const size_t NS = a.node_stride;
    T* N = a.nodes;

    if (a.phase == PH_DIAG) {
        diagnostics(a, cap, c, red);
        return;
    }

    Patch<T> P;
    P.drho = reinterpret_cast<T*>(smem);
    P.ux = P.drho + a.patch_cap;
    P.uy = P.ux + a.patch_cap;
    Scratch<T> S;
    S.px = P.uy + a.patch_cap;
    S.py = S.px + a.max_nv;
    S.qx = S.py + a.max_nv;
    S.qy = S.qx + a.max_nv;
    T* node_lds[8];
    for (int k = 0; k < 8; k++) node_lds[k] = S.qy + (size_t)(k + 1) * a.max_nv;
    S.dx = node_lds[0];
    S.dy = node_lds[1];
    S.ux = node_lds[2];
    S.uy = node_lds[3];
    S.l0 = node_lds[4];
    S.l0l = node_lds[5];
    S.ks = node_lds[6];
    S.th0 = node_lds[7];
    for (int k = 0; k < kNodeScratch; k++) S.t[k] = S.th0 + (size_t)(k + 1) * a.max_nv;

    int st = 0;
    const bool prime = (a.phase & PH_PRIME) && !cap.primed;
    const bool doB = (a.phase & PH_B) && cap.primed;
    const bool doA = (a.phase & PH_A) != 0;
    long long refx = (long long)cap.ref_x, refy = (long long)cap.ref_y;
    const bool need_field = prime || doB || (doA && DYN);
    const T gxf = (T)cap.gx;

    // The patch box of this capsule's last launch: the waves that hold no node
    // stage it while the node waves load the node state, so that the two
    // load latencies overlap.  Below, the box the nodes need is checked
    // against it; the patch is staged again if it does not fit.  (Each cell's
    // staged values do not depend on the box, so the results do not either.)
    const int node_threads = (nv + 63) / 64 * 64;
    const int4 hint = need_field ? hint0 : make_int4(0, 0, 0, 0);
    const bool early = hint.z > 0 && hint.w > 0 && (long long)hint.z * hint.w <= a.patch_cap &&
                       node_threads < nt;
    if (early && tid >= node_threads) {
        P.ox = hint.x;
        P.oy = hint.y;
        P.W = hint.z;
        P.H = hint.w;
        const int ncell = P.W * P.H, ns = nt - node_threads;
        for (int i = tid - node_threads; i < ncell; i += 3 * ns)
            stage_cells<T, 3>(a, g, P, refx, refy, gxf, i, ns);
    }

    float mn[2] = {3e38f, 3e38f}, mxv[2] = {-3e38f, -3e38f};
    bool finite = true;
    for (int v = tid; v < nv; v += nt) {
        const T x = N[NF_HX * NS + off + v], y = N[NF_HY * NS + off + v];
        S.px[v] = x;
        S.py[v] = y;
        S.qx[v] = N[NF_LX * NS + off + v];
        S.qy[v] = N[NF_LY * NS + off + v];
        S.dx[v] = N[NF_DX * NS + off + v];
        S.dy[v] = N[NF_DY * NS + off + v];
        S.ux[v] = N[NF_UX * NS + off + v];
        S.uy[v] = N[NF_UY * NS + off + v];
        S.l0[v] = N[NF_L0 * NS + off + v];
        S.l0l[v] = N[NF_L0L * NS + off + v];
        S.ks[v] = N[NF_KS * NS + off + v];
        S.th0[v] = N[NF_TH0 * NS + off + v];
        finite = finite && isfinite(x) && isfinite(y);
        mn[0] = fminf(mn[0], (float)x);
        mn[1] = fminf(mn[1], (float)y);
        mxv[0] = fmaxf(mxv[0], (float)x);
        mxv[1] = fmaxf(mxv[1], (float)y);
    }
    if (!finite) { mn[0] = -3e38f; }
    // S.px/py are visible after its first barrier.  Its closing barrier (which
    // keeps red[.][0..3] from being written again before every wave has read
    // them) is left to the staging barrier below where there is one.
    block_minmax(mn, mxv, red, !need_field);
    // Dynamic node update: the enclosed area of x^n for the membrane forces,
    // as wave partials in red[.][7], summed in wave order (as block_sum) after
    // the staging barrier below
    const bool dyn_forces = doB && DYN && !cap.rigid;
    if (dyn_forces) {
        const double acc = wave_sum(area_share(S, nv));
        if ((tid & 63) == 0) red[tid >> 6][7] = acc;
    }

    // ---- fluid patch: bounding box + 3 cells (probe 1.2 + support 1.5 + motion)
    if (need_field) {
        if (!(mn[0] > -1e30f && mxv[0] < 1e30f && mn[1] > -1e30f && mxv[1] < 1e30f)) {
            if (tid == 0) atomicOr(a.status, ST_NONFINITE);
            return;
        }
        // offsets from the reference point stay small; anything else cannot be staged
        if (!(mn[0] > -1e6f && mxv[0] < 1e6f && mn[1] > -1e6f && mxv[1] < 1e6f)) {
            if (tid == 0) atomicOr(a.status, ST_PATCH);
            return;
        }
        const int ox = (int)floorf(mn[0]) - 3, oy = (int)floorf(mn[1]) - 3;
        const int W = (int)floorf(mxv[0]) - (int)floorf(mn[0]) + 7;
        const int H = (int)floorf(mxv[1]) - (int)floorf(mn[1]) + 7;
        if (early && ox >= hint.x && oy >= hint.y && ox + W <= hint.x + hint.z &&
            oy + H <= hint.y + hint.w) {
            P.ox = hint.x;
            P.oy = hint.y;
            P.W = hint.z;
            P.H = hint.w;
        } else {
            if ((long long)W * H > a.patch_cap) {
                if (tid == 0) atomicOr(a.status, ST_PATCH);
                return;
            }
            // one spare cell on every side where it fits, so that the box
            // serves the next launches while the capsule drifts
            const bool spare = (long long)(W + 2) * (H + 2) <= a.patch_cap;
            P.ox = spare ? ox - 1 : ox;
            P.oy = spare ? oy - 1 : oy;
            P.W = spare ? W + 2 : W;
            P.H = spare ? H + 2 : H;
            // three cells per thread with all their loads in flight together
            const int ncell = P.W * P.H;
            for (int i = tid; i < ncell; i += 3 * nt) stage_cells<T, 3>(a, g, P, refx, refy, gxf, i, nt);
        }
        __syncthreads();
    }

    // ---- start-up (reading: u_v^0 = U(x^0), x^{-1} = x^0 - U(x^0))
    if (prime && cap.rigid) {
        rigid_prime(a, S, P, cap, c, st, red);
    } else if (prime) {
        for (int v = tid; v < nv; v += nt) {
            T Ux, Uy;
            interp_u(P, S.px[v], S.py[v], Ux, Uy, st);
            N[NF_UX * NS + off + v] = Ux;
            N[NF_UY * NS + off + v] = Uy;
            N[NF_DX * NS + off + v] = Ux;
            N[NF_DY * NS + off + v] = Uy;
            S.ux[v] = Ux;
            S.uy[v] = Uy;
            S.dx[v] = Ux;
            S.dy[v] = Uy;
        }
    }

    // ---- node update closing the previous step
    if (doB) {
        double csum[2] = {0.0, 0.0};
        if (cap.rigid) rigid_update(a, S, P, cap, c, st, red, csum);
        if (dyn_forces) {  // element and probe terms, t12, t13 (Eq. 23); nodal sums below
            double area = red[0][7];
            for (int w = 1; w < (int)(nt >> 6); w++) area += red[w][7];
            dynamic_forces(S, P, nv, cap.kb, cap.ka, cap.A0, 0.5 * area, (T)cap.nu, a.max_edge,
                           a.max_dA, st);
        }
        const T half_inv_m = (T)(0.5 / cap.mv);
        for (int v = cap.rigid ? nv : tid; v < nv; v += nt) {
            T Ux, Uy;  // tentative velocity, Eq. 23 (Dynamic: interpolated beside the probes)
            if (DYN) {
                Ux = S.t[12][v];
                Uy = S.t[13][v];
            } else {
                interp_u(P, S.px[v], S.py[v], Ux, Uy, st);
            }
            const T dox = S.dx[v], doy = S.dy[v];
            T dx, dy;
            if (DYN) {
                T fix, fiy, fex, fey;
                dynamic_node_forces(S, v, nv, cap.kb, fix, fiy, fex, fey);
                S.t[8][v] = fix;  // (kept for the tape of a launch without phase A)
                S.t[9][v] = fiy;
                T fx = fix + fex, fy = fiy + fey;
                if (a.contact) {
                    fx += N[NF_CX * NS + off + v];
                    fy += N[NF_CY * NS + off + v];
                }
                dx = Ux + half_inv_m * fx;  // Eq. 23
                dy = Uy + half_inv_m * fy;
                const T uvx = T(1.5) * dx - T(0.5) * dox, uvy = T(1.5) * dy - T(0.5) * doy;  // Eq. 24
                N[NF_UX * NS + off + v] = uvx;
                N[NF_UY * NS + off + v] = uvy;
                S.ux[v] = uvx;
                S.uy[v] = uvy;
                N[NF_FX * NS + off + v] = fx;
                N[NF_FY * NS + off + v] = fy;
                N[NF_EX * NS + off + v] = fex;
                N[NF_EY * NS + off + v] = fey;
            } else {
                dx = dox * T(1.0 / 3.0) + Ux * T(2.0 / 3.0);  // Eq. 25 as an increment
                dy = doy * T(1.0 / 3.0) + Uy * T(2.0 / 3.0);
            }
            if (!(fabs(dx) < T(1) && fabs(dy) < T(1))) st |= ST_MOVE;
            N[NF_DX * NS + off + v] = dx;
            S.dx[v] = dx;
            N[NF_DY * NS + off + v] = dy;
            S.dy[v] = dy;
            T hx = S.px[v], lx = S.qx[v];
            T hy = S.py[v], ly = S.qy[v];
            comp_add(hx, lx, dx);
            comp_add(hy, ly, dy);
            S.t[4][v] = hx;  // new positions, published after the barrier
            S.t[5][v] = hy;
            S.t[6][v] = lx;
            S.t[7][v] = ly;
            csum[0] += (double)hx;
            csum[1] += (double)hy;
        }
        block_sum<2>(csum, red);
        // keep the reference point within one lattice unit of the node mean
        const double mx = csum[0] / nv, my = csum[1] / nv;
        const T kx = fabs(mx) >= 1.0 ? (T)rint(mx) : T(0);
        const T ky = fabs(my) >= 1.0 ? (T)rint(my) : T(0);
        for (int v = tid; v < nv; v += nt) {
            T hx = S.t[4][v], hy = S.t[5][v], lx = S.t[6][v], ly = S.t[7][v];
            if (kx != T(0) || ky != T(0)) {
                comp_add(hx, lx, -kx);
                comp_add(hy, ly, -ky);
            }
            S.px[v] = hx;
            S.py[v] = hy;
            S.qx[v] = lx;
            S.qy[v] = ly;
            N[NF_HX * NS + off + v] = hx;
            N[NF_HY * NS + off + v] = hy;
            N[NF_LX * NS + off + v] = lx;
            N[NF_LY * NS + off + v] = ly;
        }
        if (kx != T(0) || ky != T(0)) {
            cap.ref_x += (double)kx;
            cap.ref_y += (double)ky;
            refx += (long long)kx;
            refy += (long long)ky;
            P.ox -= (int)kx;
            P.oy -= (int)ky;
            if (tid == 0) {
                a.caps[c].ref_x = cap.ref_x;
                a.caps[c].ref_y = cap.ref_y;
            }
        }
        __syncthreads();
    }

    // ---- near region of this step's grid update (overlapped schedule): the
    // bounding box of x^n and x^{n-1} = x^n - d^n plus 5 cells covers the
    // supports of F^n and F^{n-1} and the patch the next IB launch stages
    if (a.rects) {
        float nmn[2] = {3e38f, 3e38f}, nmx[2] = {-3e38f, -3e38f};
        for (int v = tid; v < nv; v += nt) {
            const float x = (float)S.px[v], y = (float)S.py[v];
            const float xo = (float)(S.px[v] - S.dx[v]), yo = (float)(S.py[v] - S.dy[v]);
            nmn[0] = fminf(nmn[0], fminf(x, xo));
            nmn[1] = fminf(nmn[1], fminf(y, yo));
            nmx[0] = fmaxf(nmx[0], fmaxf(x, xo));
            nmx[1] = fmaxf(nmx[1], fmaxf(y, yo));
        }
        block_minmax(nmn, nmx, red);
        NearRect r;
        r.x0 = (int)(refx + (long long)floorf(nmn[0])) - 5;
        r.x1 = (int)(refx + (long long)floorf(nmx[0])) + 5;
        r.y0 = (int)(refy + (long long)floorf(nmn[1])) - 5;
        r.y1 = (int)(refy + (long long)floorf(nmx[1])) + 5;
        if (tid == 0) a.rects[c] = r;
        const RectUnits u = rect_units(r, g);
        const int units = u.nrows * u.nsegs;
        for (int q = tid; q < units; q += nt) {
            const int ri = q / u.nsegs, si = q - ri * u.nsegs;
            int y = u.ry0 + ri;
            if (y >= g.ny) y -= g.ny;
            const int seg = si < u.nA ? u.sa + si : si - u.nA;
            a.near_map[y * g.nseg + seg] = a.stamp;
        }
    }

    // ---- forcing of the new step
    if (doA) {
        if (DYN) {
            for (int v = tid; v < nv; v += nt) {
                const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
                int cx, cy;
                T phi[9];
                mls<T, false>(S.px[v], S.py[v], cx, cy, phi, nullptr, nullptr);
                T Ux = T(0), Uy = T(0);  // Eq. 8
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    int idx;
                    if (!patch_index(P, cx, cy, k, idx)) { st |= ST_PATCH; continue; }
                    if (isnan(P.drho[idx])) { st |= ST_WALL; continue; }
                    Ux += phi[k] * P.ux[idx];
                    Uy += phi[k] * P.uy[idx];
                }
                const T Fx = S.ux[v] - Ux;  // (U_b - U) / dt, step 1
                const T Fy = S.uy[v] - Uy;
                T ax, ay, bx, by;
                edge(S, vl, v, ax, ay);
                edge(S, v, vr, bx, by);
                const T cv = T(0.5) * (sqrt(ax * ax + ay * ay) + sqrt(bx * bx + by * by));
                cache_weights(S, v, cx, cy, phi);
                S.t[8][v] = cv * Fx;
                S.t[9][v] = cv * Fy;
            }
        } else {
            kinematic_forces(S, nv, cap.kb, cap.ka, cap.A0, red, a.max_edge, a.max_dA, st);
            for (int v = tid; v < nv; v += nt) {
                T fx, fy;
                membrane_node_force(S, v, nv, cap.kb, fx, fy);
                if (a.contact) {
                    fx += N[NF_CX * NS + off + v];
                    fy += N[NF_CY * NS + off + v];
                }
                S.t[8][v] = fx;
                S.t[9][v] = fy;
                N[NF_FX * NS + off + v] = fx;
                N[NF_FY * NS + off + v] = fy;
            }
        }
        __syncthreads();
        // pre-sum in LDS where the staged patch box holds the sums (fewer
        // global atomics: 388 capsules 42.7 -> 30.0 us per launch, 32 capsules
        // 25.2 -> 24.3 us; a lone capsule pays about 0.3 us for the barriers)
        if (need_field && (size_t)P.W * P.H * 20 <= (size_t)3 * a.patch_cap * sizeof(T))
            spread_patch(a, g, S, P, nv, refx, refy, st);
        else
            spread_cached(a, g, S, nv, refx, refy, st);
    }
    if (prime && tid == 0) a.caps[c].primed = 1;
    if (need_field && a.hints && tid == 0) a.hints[c] = make_int4(P.ox, P.oy, P.W, P.H);
    // trajectory tape (reverse sweeps): the node state of this time level
    if (a.tape_nodes) {
        T* TN = a.tape_nodes;
        for (int v = tid; v < nv; v += nt) {
            TN[NF_HX * NS + off + v] = S.px[v];
            TN[NF_HY * NS + off + v] = S.py[v];
            TN[NF_LX * NS + off + v] = S.qx[v];
            TN[NF_LY * NS + off + v] = S.qy[v];
            TN[NF_DX * NS + off + v] = S.dx[v];
            TN[NF_DY * NS + off + v] = S.dy[v];
            TN[NF_UX * NS + off + v] = S.ux[v];
            TN[NF_UY * NS + off + v] = S.uy[v];
            TN[kTapeFX * NS + off + v] = S.t[8][v];  // c_v F_v spread in phase A
            TN[kTapeFY * NS + off + v] = S.t[9][v];
        }
        if (tid == 0) {
            a.tape_ref[2 * c] = cap.ref_x;
            a.tape_ref[2 * c + 1] = cap.ref_y;
        }
    }
    if (st) atomicOr(a.status, st);
}

// One instance per coupling (DYN = a0.dynamic): each holds only its own
// scheme's phases, which keeps the code a launch runs together.
//
// Two register budgets per coupling.  Beside the far pass of a split step
// an IB block must stay within 112 VGPRs per lane, so that it
// shares a compute unit with seven far waves per SIMD; the compiler's own
// allocation for this kernel is 106 VGPRs, with 118-145 SGPRs spilled to
// VGPR lanes.  Launched alone (the serial schedule, batches, diagnostics) it
// runs faster with more registers: the WIDE instance opens with s_setprio 0,
// the default wave priority, so nothing changes at run time, but with it at
// the entry this compiler allocates 151 VGPRs and spills half as many SGPRs.
// Measured per step: 1024x256 channel 24.1 -> 23.7 us, 2048x512 channel with
// 32 capsules 33.5 -> 33.1 us.  At 151 VGPRs one block fills a compute
// unit's register file, so the wide instance serves only launches that run
// alone with at most one block per compute unit; beside the far pass a build
// with that allocation took 190 us against 80 us and slowed the 4096^2 step by
// 11 us, and the 388-capsule ensemble's launch took 36 us against 27 us.
template <typename T, bool DYN, bool WIDE>
__global__ __launch_bounds__(kIBThreads) void k_ib(IBArgs<T> a0)
{
    if (WIDE) __builtin_amdgcn_s_setprio(0);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kIBThreads / 64][8];
    ib_block<T, DYN>(a0, smem, red);  // every exit of ib_block is block-uniform
    if (a0.done_count) {
        // the block's stores (near map, force level, node state) are made
        // visible device-wide before the count announces them
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(a0.done_count, 1ull);
        }
    }
}

template <typename T>
size_t ib_lds_bytes(int patch_cap, int max_nv)
{
    return sizeof(T) * ((size_t)3 * patch_cap + (size_t)kNodeLdsArrays * max_nv);
}

template <typename T>
hipError_t ib_set_lds_limit(size_t bytes)
{
    const void* fns[4] = {reinterpret_cast<const void*>(&k_ib<T, true, false>),
                          reinterpret_cast<const void*>(&k_ib<T, false, false>),
                          reinterpret_cast<const void*>(&k_ib<T, true, true>),
                          reinterpret_cast<const void*>(&k_ib<T, false, true>)};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_ib(const IBArgs<T>& a, int ncap, size_t lds_bytes, hipStream_t s, bool wide)
{
    if (ncap <= 0) return hipSuccess;
    const dim3 grid(ncap), block(kIBThreads);
    if (!wide) {
        if (a.dynamic)
            hipLaunchKernelGGL((k_ib<T, true, false>), grid, block, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_ib<T, false, false>), grid, block, lds_bytes, s, a);
    } else {
        if (a.dynamic)
            hipLaunchKernelGGL((k_ib<T, true, true>), grid, block, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_ib<T, false, true>), grid, block, lds_bytes, s, a);
    }
    return hipGetLastError();
}

// Spreading of a taped step: each node's taped force c_v F_v with the MLS
// weights at its taped position, relative to the taped reference point, into
// the step's force level.  These are the contributions, in fixed point, of
// the IB launch that wrote the tape (same weights, same products), so the
// level matches it bit for bit.  One block per capsule, one thread per node.
template <typename T>
__global__ __launch_bounds__(kIBThreads) void k_spread_tape(SpreadTapeArgs<T> a)
{
    const int c = blockIdx.x;
    const CapsuleDev cap = a.caps[c];
    GridArgs g;
    g.nx = cap.nx;
    g.ny = cap.ny;
    g.nxp = cap.nxp;
    g.nseg = cap.nseg;
    g.periodic_y = cap.periodic_y;
    g.periodic_x = cap.periodic_x;
    IBArgs<T> ia;
    ia.fib_next = a.fib + cap.fib_off;
    ia.flags_next = a.flags + cap.flag_off;
    const long long refx = (long long)a.ref[2 * c], refy = (long long)a.ref[2 * c + 1];
    const size_t NS = a.node_stride;
    const int off = cap.node_offset;
    const T* TN = a.tape;
    int st = 0;
    const SpreadRef r = spread_ref(g, refx, refy);
    for (int v = threadIdx.x; v < cap.nv; v += blockDim.x) {
        int cx, cy;
        T phi[9];
        mls<T, false>(TN[NF_HX * NS + off + v], TN[NF_HY * NS + off + v], cx, cy, phi, nullptr,
                      nullptr);
        const T fx = TN[kTapeFX * NS + off + v], fy = TN[kTapeFY * NS + off + v];
#pragma unroll
        for (int k = 0; k < 9; k++) spread_one(ia, g, r, cx, cy, k, phi[k] * fx, phi[k] * fy, st);
    }
    if (st) atomicOr(a.status, st);
}

template <typename T>
hipError_t launch_spread_tape(const SpreadTapeArgs<T>& a, int ncap, hipStream_t s)
{
    if (ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spread_tape<T>, dim3(ncap), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- contact
// World bounding box of each capsule's current nodes (one block per capsule).
template <typename T>
__global__ __launch_bounds__(kIBThreads) void k_bounds(ContactArgs<T> a)
{
    __shared__ double red[kIBThreads / 64][8];
    const int c = blockIdx.x;
    const CapsuleDev cap = a.caps[c];
    const size_t NS = a.node_stride;
    const T* N = a.nodes;
    float mn[2] = {3e38f, 3e38f}, mx[2] = {-3e38f, -3e38f};
    for (int v = threadIdx.x; v < cap.nv; v += blockDim.x) {
        const float x = (float)N[NF_HX * NS + cap.node_offset + v];
        const float y = (float)N[NF_HY * NS + cap.node_offset + v];
        mn[0] = fminf(mn[0], x);
        mn[1] = fminf(mn[1], y);
        mx[0] = fmaxf(mx[0], x);
        mx[1] = fmaxf(mx[1], y);
    }
    block_minmax(mn, mx, red);
    if (threadIdx.x == 0)
        a.bounds[c] = make_float4((float)cap.ref_x + mn[0], (float)cap.ref_y + mn[1],
                                  (float)cap.ref_x + mx[0], (float)cap.ref_y + mx[1]);
}

// Eq. 27 (Sec. 3.4): node v of capsule c, at distance d < cutoff from a node
// of another capsule of the same lattice, receives (1e-4 / (8 sqrt 2))
// sqrt(1 / d^5) (dx = 1) along its inward normal, summed over those nodes.
// The inward normal is minus the normalized sum of the outward normals of the
// node's two elements.  Distances take the nearest periodic image.  One
// block per capsule; capsules whose boxes (grown by the cutoff) miss this
// one's are skipped, the others are staged in LDS.  FP64.
// The pairs (node of this capsule, node of the other) are dealt to
// K = min(nt / nv, kContactGroups) groups of nv threads: thread t takes node
// t % nv against every K-th node of the other capsule from t / nv on, and the
// K partial sums of a node are added in group order (fixed, so runs repeat bit
// for bit).  The other capsules' records are staged in LDS in chunks, and
// each capsule is staged at the periodic image nearest to this one, so that a
// pair's own image needs the division only where |dx| still exceeds half the
// period (below it the rounded quotient is 0); the root and the force only for
// pairs whose squared distance is below the cutoff's.
template <typename T>
__global__ __launch_bounds__(kIBThreads) void k_contact(ContactArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const CapsuleDev cap = a.caps[c];
    const int nv = cap.nv, off = cap.node_offset;
    const size_t NS = a.node_stride;
    const T* N = a.nodes;
    double* X = reinterpret_cast<double*>(smem);
    double* Y = X + a.max_nv;
    double* IX = Y + a.max_nv;  // inward normal
    double* IY = IX + a.max_nv;
    double* FX = IY + a.max_nv;
    double* FY = FX + a.max_nv;
    double* BX = FY + a.max_nv;  // the other capsule, in this capsule's frame
    double* BY = BX + a.max_nv;
    double* PX = BY + a.max_nv;  // per-thread partial sums, nt each
    double* PY = PX + nt;
    for (int v = tid; v < nv; v += nt) {
        X[v] = (double)N[NF_HX * NS + off + v] + (double)N[NF_LX * NS + off + v];
        Y[v] = (double)N[NF_HY * NS + off + v] + (double)N[NF_LY * NS + off + v];
        FX[v] = FY[v] = 0.0;
    }
    __syncthreads();
    for (int v = tid; v < nv; v += nt) {
        const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
        const double ax = X[v] - X[vl], ay = Y[v] - Y[vl];
        const double bx = X[vr] - X[v], by = Y[vr] - Y[v];
        const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
        const double nx = ay / la + by / lb, ny = -ax / la - bx / lb;
        const double nn = sqrt(nx * nx + ny * ny);
        IX[v] = -nx / nn;
        IY[v] = -ny / nn;
    }
    const float4 me = a.bounds[c];
    const double Lx = cap.nx, Ly = cap.ny;
    const double C = 1e-4 / (8.0 * sqrt(2.0));
    const float cut = (float)a.cutoff;
    // squared-distance screen, a little wider than the cutoff: every pair the
    // exact test below accepts passes it
    const double cut2 = a.cutoff * a.cutoff * (1.0 + 1e-6);
    const int K = nv > 0 ? max(1, min(nt / nv, kContactGroups)) : 1;
    const int vq = nv > 0 ? tid % nv : 0, kq = nv > 0 ? tid / nv : 0;
    // the other capsules' records, kContactChunk at a time, one per thread
    // (their loads in flight together, not one dependent load per capsule)
    __shared__ float4 s_box[kContactChunk];
    __shared__ double s_rx[kContactChunk], s_ry[kContactChunk];
    __shared__ int s_nv[kContactChunk], s_off[kContactChunk], s_inst[kContactChunk];
    for (int o0 = 0; o0 < a.ncap; o0 += kContactChunk) {
        const int m = min(kContactChunk, a.ncap - o0);
        __syncthreads();  // the last chunk's records are read no more
        if (tid < m) {
            const CapsuleDev& r = a.caps[o0 + tid];
            s_box[tid] = a.bounds[o0 + tid];
            s_rx[tid] = r.ref_x;
            s_ry[tid] = r.ref_y;
            s_nv[tid] = r.nv;
            s_off[tid] = r.node_offset;
            s_inst[tid] = r.inst;
        }
        __syncthreads();
        for (int q = 0; q < m; q++) {
            const int o = o0 + q;
            if (o == c || s_inst[q] != cap.inst) continue;
            const float4 ob = s_box[q];
            const int onv = s_nv[q], ooff = s_off[q];
            // box test with the nearest periodic image in x (and y when periodic)
            float sx = (0.5f * (ob.x + ob.z)) - (0.5f * (me.x + me.z));
            const float ix = cap.periodic_x ? rintf(sx / (float)Lx) : 0.0f;
            sx -= (float)Lx * ix;
            float sy = (0.5f * (ob.y + ob.w)) - (0.5f * (me.y + me.w));
            const float iy = cap.periodic_y ? rintf(sy / (float)Ly) : 0.0f;
            sy -= (float)Ly * iy;
            const float hx = 0.5f * ((ob.z - ob.x) + (me.z - me.x)) + cut;
            const float hy = 0.5f * ((ob.w - ob.y) + (me.w - me.y)) + cut;
            if (fabsf(sx) > hx || fabsf(sy) > hy) continue;
            __syncthreads();
            // staged at the periodic image nearest to this capsule (box centres),
            // so that the pair loop rarely needs the image division
            const double rx = s_rx[q] - cap.ref_x - (double)ix * Lx;
            const double ry = s_ry[q] - cap.ref_y - (double)iy * Ly;
            for (int j = tid; j < onv; j += nt) {
                BX[j] = rx + (double)N[NF_HX * NS + ooff + j] + (double)N[NF_LX * NS + ooff + j];
                BY[j] = ry + (double)N[NF_HY * NS + ooff + j] + (double)N[NF_LY * NS + ooff + j];
            }
            __syncthreads();
            // the force on node v from nodes j0, j0 + step, ... of the other capsule
            auto pair_sum = [&](int v, int j0, int step, double& fx, double& fy) {
                const double xv = X[v], yv = Y[v];
                for (int j = j0; j < onv; j += step) {
                    double dx = BX[j] - xv, dy = BY[j] - yv;
                    if (cap.periodic_x && fabs(dx) > 0.5 * Lx) dx -= Lx * rint(dx / Lx);
                    if (cap.periodic_y && fabs(dy) > 0.5 * Ly) dy -= Ly * rint(dy / Ly);
                    const double d2 = dx * dx + dy * dy;
                    if (d2 < cut2) {
                        const double d = sqrt(d2);
                        if (d < a.cutoff && d > 0.0) {
                            const double mag = C * sqrt(1.0 / (d * d * d * d * d));
                            fx += mag * IX[v];
                            fy += mag * IY[v];
                        }
                    }
                }
            };
            if (K == 1) {
                for (int v = tid; v < nv; v += nt) {
                    double fx = 0.0, fy = 0.0;
                    pair_sum(v, 0, 1, fx, fy);
                    FX[v] += fx;
                    FY[v] += fy;
                }
            } else {
                double fx = 0.0, fy = 0.0;
                if (kq < K) pair_sum(vq, kq, K, fx, fy);
                PX[tid] = fx;
                PY[tid] = fy;
                __syncthreads();
                for (int v = tid; v < nv; v += nt) {
                    double sx = 0.0, sy = 0.0;
                    for (int k = 0; k < K; k++) {
                        sx += PX[v + k * nv];
                        sy += PY[v + k * nv];
                    }
                    FX[v] += sx;
                    FY[v] += sy;
                }
            }
        }
    }
    T* W = a.nodes;
    for (int v = tid; v < nv; v += nt) {
        W[NF_CX * NS + off + v] = (T)FX[v];
        W[NF_CY * NS + off + v] = (T)FY[v];
    }
}

template <typename T>
hipError_t contact_set_lds_limit(int max_nv)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_contact<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(contact_lds_bytes(max_nv)));
}

template <typename T>
hipError_t launch_contact(const ContactArgs<T>& a, hipStream_t s)
{
    if (a.ncap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bounds<T>, dim3(a.ncap), dim3(kIBThreads), 0, s, a);
    hipLaunchKernelGGL(k_contact<T>, dim3(a.ncap), dim3(kIBThreads),
                       contact_lds_bytes(a.max_nv), s, a);
    return hipGetLastError();
}

// ------------------------------------------------------- state transfers

template <typename T>
__global__ void k_get_pop_plane(const T* src, double* out, int plane, int unshift, GridArgs g)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    T s[9];
    pull(src, x, y, g, (T)g.gx, s);
    T v = s[0];
#pragma unroll
    for (int i = 1; i < 9; i++)
        if (i == plane) v = s[i];
    double d = (double)v + ref_first<T>(g, plane, y);
    if (unshift) d += plane == 0 ? 4.0 / 9.0 : (plane < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    out[(size_t)y * g.nx + x] = d;
}

template <typename T>
hipError_t launch_get_pop_plane(const T* src, double* out, int plane, int unshift,
                                const GridArgs& g, hipStream_t s)
{
    hipLaunchKernelGGL(k_get_pop_plane<T>, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, src,
                       out, plane, unshift, g);
    return hipGetLastError();
}

// f*_i(x) = f^n_i(x + e_i): the pull of the next step then returns f^n.
template <typename T>
__global__ void k_set_pop_plane(T* dst, const double* in, int plane, GridArgs g)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    int xd = x + kEx[plane];
    xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
    int yd = y + kEy[plane];
    if (g.periodic_y) yd = yd < 0 ? yd + g.ny : (yd >= g.ny ? yd - g.ny : yd);
    else if (yd < 0 || yd >= g.ny) return;
    const double w = plane == 0 ? 4.0 / 9.0 : (plane < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    dst[(size_t)plane * g.ny * g.nxp + (size_t)y * g.nxp + x] =
        (T)(in[(size_t)yd * g.nx + xd] - w - ref_first<T>(g, plane, y));
}

template <typename T>
hipError_t launch_set_pop_plane(T* dst, const double* in, int plane, const GridArgs& g,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_set_pop_plane<T>, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, dst,
                       in, plane, g);
    return hipGetLastError();
}

template <typename T>
__global__ void k_get_moments(const T* src, const long long* fib, double* out, GridArgs g)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    const size_t cell = (size_t)y * g.nxp + x;
    const double Fx = g.gx + (double)fib[2 * cell] * kFixInv;
    const double Fy = (double)fib[2 * cell + 1] * kFixInv;
    T s[9];
    pull(src, x, y, g, (T)Fx, s);
    double drho = 0, jx = 0, jy = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        drho += (double)s[i];
        jx += (double)s[i] * kEx[i];
        jy += (double)s[i] * kEy[i];
    }
    const double rho = 1.0 + drho;
    const size_t plane = (size_t)g.nx * g.ny, o = (size_t)y * g.nx + x;
    out[o] = rho;
    out[plane + o] = (g.uref_c * (double)(y * (g.ny - 1 - y)) + jx + 0.5 * Fx) / rho;
    out[2 * plane + o] = (jy + 0.5 * Fy) / rho;
}

template <typename T>
hipError_t launch_get_moments(const T* src, const long long* fib, double* out, const GridArgs& g,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_get_moments<T>, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, src, fib,
                       out, g);
    return hipGetLastError();
}

__global__ void k_get_force(const long long* fib, double* out, GridArgs g)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= g.nx) return;
    const size_t cell = (size_t)y * g.nxp + x;
    const size_t plane = (size_t)g.nx * g.ny, o = (size_t)y * g.nx + x;
    out[o] = g.gx + (double)fib[2 * cell] * kFixInv;
    out[plane + o] = (double)fib[2 * cell + 1] * kFixInv;
}

hipError_t launch_get_force(const long long* fib, double* out, const GridArgs& g, hipStream_t s)
{
    hipLaunchKernelGGL(k_get_force, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, fib, out, g);
    return hipGetLastError();
}

// what: 4 x^n, 5 x^{n-1}, 6 u_v^n, 7 last nodal force, 8 all three stacked
template <typename T>
__global__ void k_get_nodes(const T* N, const CapsuleDev* caps, int c, int nv, int NS, int what,
                            double* out)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const CapsuleDev cap = caps[c];
    const int j = cap.node_offset + v;
    const size_t S = NS;
    const double x = cap.ref_x + ((double)N[NF_HX * S + j] + (double)N[NF_LX * S + j]);
    const double y = cap.ref_y + ((double)N[NF_HY * S + j] + (double)N[NF_LY * S + j]);
    const double px = x - (double)N[NF_DX * S + j], py = y - (double)N[NF_DY * S + j];
    const double ux = N[NF_UX * S + j], uy = N[NF_UY * S + j];
    if (what == 4 || what == 8) { out[2 * v] = x; out[2 * v + 1] = y; }
    double* o = what == 8 ? out + 2 * nv : out;
    if (what == 5 || what == 8) { o[2 * v] = px; o[2 * v + 1] = py; }
    o = what == 8 ? out + 4 * nv : out;
    if (what == 6 || what == 8) { o[2 * v] = ux; o[2 * v + 1] = uy; }
    if (what == 7) { out[2 * v] = N[NF_FX * S + j]; out[2 * v + 1] = N[NF_FY * S + j]; }
}

template <typename T>
hipError_t launch_get_nodes(const T* nodes, const CapsuleDev* caps, int cap, int nv,
                            int node_stride, int what, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_get_nodes<T>, dim3((nv + 255) / 256), dim3(256), 0, s, nodes, caps, cap, nv,
                       node_stride, what, out);
    return hipGetLastError();
}

template <typename T>
__global__ void k_set_nodes(T* N, CapsuleDev* caps, int c, int nv, int NS, const double* in)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const CapsuleDev cap = caps[c];
    const int j = cap.node_offset + v;
    const size_t S = NS;
    const double rx = in[2 * v] - cap.ref_x, ry = in[2 * v + 1] - cap.ref_y;
    const T hx = (T)rx, hy = (T)ry;
    N[NF_HX * S + j] = hx;
    N[NF_HY * S + j] = hy;
    N[NF_LX * S + j] = (T)(rx - (double)hx);
    N[NF_LY * S + j] = (T)(ry - (double)hy);
    N[NF_DX * S + j] = (T)(in[2 * v] - in[2 * nv + 2 * v]);
    N[NF_DY * S + j] = (T)(in[2 * v + 1] - in[2 * nv + 2 * v + 1]);
    N[NF_UX * S + j] = (T)in[4 * nv + 2 * v];
    N[NF_UY * S + j] = (T)in[4 * nv + 2 * v + 1];
    if (v == 0) caps[c].primed = 1;
}

template <typename T>
hipError_t launch_set_nodes(T* nodes, CapsuleDev* caps, int cap, int nv, int node_stride,
                            const double* in, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_nodes<T>, dim3((nv + 255) / 256), dim3(256), 0, s, nodes, caps, cap, nv,
                       node_stride, in);
    return hipGetLastError();
}

// ---- explicit instantiations
#define LBIB_INST(T)                                                                              \
    template hipError_t launch_init<T>(T*, const GridArgs&, int, double, double, double,          \
                                       hipStream_t);                                              \
    template hipError_t launch_grid_step<T>(const T*, T*, const long long*, const int*,           \
                                            long long*, int*, const GridArgs&, hipStream_t);      \
    template hipError_t launch_grid_step_batch<T>(const T*, T*, const long long*, const int*,     \
                                                  long long*, int*, const InstDev*, const int2*,  \
                                                  int, int, int, int, bool, const int*, int,      \
                                                  int*, hipStream_t);                             \
    template hipError_t launch_grid_far<T>(const T*, T*, const long long*, const int*,            \
                                           long long*, int*, const int*, int, int*,               \
                                           const GridArgs&, hipStream_t, hipEvent_t,              \
                                           const unsigned long long*, unsigned long long);             \
    template hipError_t launch_grid_near<T>(const T*, T*, const long long*, const int*,           \
                                            long long*, int*, const NearRect*, const CapsuleDev*, \
                                            const InstDev*, int, hipStream_t);                    \
    template hipError_t launch_contact<T>(const ContactArgs<T>&, hipStream_t);                   \
    template hipError_t launch_spread_tape<T>(const SpreadTapeArgs<T>&, int, hipStream_t);         \
    template hipError_t contact_set_lds_limit<T>(int);                                            \
    template hipError_t launch_ib<T>(const IBArgs<T>&, int, size_t, hipStream_t, bool);                 \
    template size_t ib_lds_bytes<T>(int, int);                                                    \
    template hipError_t ib_set_lds_limit<T>(size_t);                                              \
    template hipError_t launch_get_pop_plane<T>(const T*, double*, int, int, const GridArgs&,     \
                                                hipStream_t);                                     \
    template hipError_t launch_set_pop_plane<T>(T*, const double*, int, const GridArgs&,          \
                                                hipStream_t);                                     \
    template hipError_t launch_get_moments<T>(const T*, const long long*, double*,                \
                                              const GridArgs&, hipStream_t);                      \
    template hipError_t launch_get_nodes<T>(const T*, const CapsuleDev*, int, int, int, int,      \
                                            double*, hipStream_t);                                \
    template hipError_t launch_set_nodes<T>(T*, CapsuleDev*, int, int, int, const double*,        \
                                            hipStream_t);

LBIB_INST(float)
LBIB_INST(double)

}  // namespace lbib
