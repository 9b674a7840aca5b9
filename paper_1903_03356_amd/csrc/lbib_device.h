// Device helpers shared by the forward kernels and their reverse (adjoint)
// kernels: the D2Q9 lattice, the BGK + forcing relaxation, the pull with the
// Zou-He walls, and the staging of a capsule's fluid patch.
#pragma once

#include "lbib_internal.h"

#include <math.h>

namespace lbib {

// ------------------------------------------------------------------ lattice
// Eq. 3 velocities in the order rest, E, N, W, S, NE, NW, SW, SE.
__device__ constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <typename T>
__device__ __forceinline__ T lat_w(int i)
{
    return i == 0 ? T(4.0 / 9.0) : (i < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

template <typename T>
__device__ __forceinline__ T fix_to_real(long long v)
{
    return (T)v * (T)kFixInv;
}

// First-order weights 3 w_i of the equilibrium and forcing terms.  3 w_axis is
// the rounded 1/3 and 3 w_diag is chosen as (1 - 2 * 3 w_axis) / 4, so that
// 2 (3 w_axis) + 4 (3 w_diag) = 1 exactly in binary: the first moment of the
// equilibrium then returns the momentum exactly instead of (1 + 7e-9) times it,
// a bias that would otherwise add up coherently over a channel flow in FP32.
template <typename T>
struct FirstOrderW {
    static constexpr T axis = T(1.0 / 3.0);
    static constexpr T diag = (T(1) - T(2) * axis) / T(4);
};

// Stored populations: slot i at a node of row y holds
//   f_i - w_i - (3 w_i) e_ix u_ref(y),
// the deviation from the rest weights and from the first-order term of the
// equilibrium of a reference flow along x, u_ref(y) = uref_c y (H - y)
// (H = ny - 1): the Poiseuille profile a periodic channel starts from, 0 for
// every other lattice.  In a channel the stored values are then the
// non-equilibrium and second-order parts (about 1e-4) instead of the whole
// first-order term (about 1e-2), so the FP32 rounding of every store is about
// a hundred times finer; in a steady flow each store rounds the same way at
// every step, and at the coarser scale those roundings add up to a drift of
// 1e-5 of the velocity over 2e4 steps.  (3 w_i) are the first-order weights
// above, whose moments give u_ref back exactly.
template <typename T>
__device__ __forceinline__ T uref_at(const GridArgs& g, int y)
{
    return (T)g.uref_c * (T)(y * (g.ny - 1 - y));
}

// A population pulled from row y - e_iy to row y changes reference:
// d_i = stored_i + (3 w_i) e_ix (u_ref(y - e_iy) - u_ref(y)), nonzero for the
// four diagonals only: dm = (3 w_d)(u_ref(y - 1) - u_ref(y)) =
// (3 w_d) uref_c (2y - H - 1) and dp = (3 w_d)(u_ref(y + 1) - u_ref(y)) =
// (3 w_d) uref_c (H - 2y - 1), in the population type (the integer factors
// are exact there; the offsets are about 1e-6 and carry a rounding of 1e-13).
// Without a reference they are +0, which leaves every value unchanged; adding
// them unconditionally measured no slower than a branch around them.
template <typename T>
__device__ __forceinline__ void add_pull_offsets(const GridArgs& g, int y, T s[9])
{
    const T c3 = (T)((double)FirstOrderW<T>::diag * g.uref_c);
    const T dm = c3 * (T)(2 * y - g.ny);
    const T dp = c3 * (T)(g.ny - 2 - 2 * y);
    s[5] += dm;
    s[6] -= dm;
    s[7] -= dp;
    s[8] += dp;
}

// BGK relaxation with the forcing term for one direction, deviation form:
// s* = s - omega (s - (f_eq - r)) + (1 - omega/2) w [3 (e - u).F + 9 (e.u)(e.F)]
// with r = w + 3 w e.u_ref the reference of the stored values and
// f_eq - r = w (rho - 1) + 3 w (e . (m - u_ref)) + w rho (4.5 (e.u)^2 - 1.5 u^2),
// m - u_ref = sum s e + F/2 taken as is (em), so that rho * (m / rho) rounding
// does not leak into the momentum; u = m / rho.
template <typename T>
__device__ __forceinline__ T relax(T s, T w, T w3, T eu, T em, T eF, T drho, T rho, T usq15,
                                   T uF, T om, T pre)
{
    const T seq = w * drho + w3 * em + w * rho * (T(4.5) * eu * eu - usq15);
    const T src = pre * (w3 * eF + w * (T(9) * eu * eF - T(3) * uF));
    return s - om * (s - seq) + src;
}

// Population loads of the pull.  The lines of the three directions with
// e_x = 0 (rest, north, south) are read by one wave only, so they are loaded
// as streaming (non-temporal) reads and leave the L2 to the lines of the
// x-shifted directions, which the neighbouring segment's wave reads too.
// Measured on a 4096 x 4096 pass: streaming the three e_x = 0 loads 2 % faster
// than plain loads, streaming all nine 0.5 % slower.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p)
{
    return __builtin_nontemporal_load(p);
}

// Raw pull of the nine populations arriving at an interior node.
template <typename T>
__device__ __forceinline__ void pull_interior(const T* __restrict__ src, int x, int y,
                                              const GridArgs& g, T s[9])
{
    const size_t plane = (size_t)g.ny * g.nxp;
    const size_t r0 = (size_t)y * g.nxp, rm = (size_t)(y - 1) * g.nxp, rp = (size_t)(y + 1) * g.nxp;
    s[0] = ld_stream(&src[r0 + x]);
    s[1] = src[plane + r0 + x - 1];
    s[2] = ld_stream(&src[2 * plane + rm + x]);
    s[3] = src[3 * plane + r0 + x + 1];
    s[4] = ld_stream(&src[4 * plane + rp + x]);
    s[5] = src[5 * plane + rm + x - 1];
    s[6] = src[6 * plane + rm + x + 1];
    s[7] = src[7 * plane + rp + x + 1];
    s[8] = src[8 * plane + rp + x - 1];
}

// Open channel (Sec. 3.2): Zou-He velocity inlet at x = 0 with the parabolic
// profile u_x = 4 u_max y (H - y) / H^2, u_y = 0 (f1, f5, f8 unknown), and
// Zou-He pressure outlet at x = nx - 1 with rho = rho_out, u_y = 0 (f3, f6, f7
// unknown); no force acts on these columns.  Corners (u = 0): each unknown
// opposite a known population takes it, the two buried diagonal populations
// share the mass deficit, with the density of the inner diagonal neighbour at
// this time level.  Deviation form: the known weights sum to 1, so the
// textbook formulas keep their shape with 1 + sum(s) for sum(f).
template <typename T>
__device__ __forceinline__ void open_boundary(const T* __restrict__ src, int x, int y,
                                              const GridArgs& g, T s[9])
{
    // Every case below sets all of n1..n8 (the untouched ones to themselves),
    // so that the branches store to the same slots of s and s stays in
    // registers (stores to different slots get merged into one with a computed
    // index, which puts s in scratch memory).
    T n1 = s[1], n2 = s[2], n3 = s[3], n4 = s[4], n5 = s[5], n6 = s[6], n7 = s[7], n8 = s[8];
    const bool bot = y == 0, top = y == g.ny - 1;
    if (bot || top) {
        T h[9];
        pull_interior(src, x == 0 ? 1 : g.nx - 2, bot ? 1 : g.ny - 2, g, h);
        const T drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
        if (x == 0 && bot) {
            n1 = n3;
            n2 = n4;
            n5 = n7;
            n6 = n8 = T(0.5) * (drho - (s[0] + n1 + n2 + n3 + n4 + n5 + n7));
        } else if (x == 0) {
            n1 = n3;
            n4 = n2;
            n8 = n6;
            n5 = n7 = T(0.5) * (drho - (s[0] + n1 + n2 + n3 + n4 + n6 + n8));
        } else if (bot) {
            n3 = n1;
            n2 = n4;
            n6 = n8;
            n5 = n7 = T(0.5) * (drho - (s[0] + n1 + n2 + n3 + n4 + n6 + n8));
        } else {
            n3 = n1;
            n4 = n2;
            n7 = n5;
            n6 = n8 = T(0.5) * (drho - (s[0] + n1 + n2 + n3 + n4 + n5 + n7));
        }
    } else {
        const T H = (T)(g.ny - 1);
        if (x == 0) {
            const T ux = T(4) * (T)g.u_in * (T)y * (H - (T)y) / (H * H);
            const T rho = (T(1) + s[0] + n2 + n4 + T(2) * (n3 + n6 + n7)) / (T(1) - ux);
            const T m = rho * ux;
            n1 = n3 + T(2.0 / 3.0) * m;
            n5 = n7 - T(0.5) * (n2 - n4) + m * T(1.0 / 6.0);
            n8 = n6 + T(0.5) * (n2 - n4) + m * T(1.0 / 6.0);
        } else {
            const T ro = (T)g.rho_out;
            const T uo = (T(1) + s[0] + n2 + n4 + T(2) * (n1 + n5 + n8)) / ro - T(1);
            const T m = ro * uo;
            n3 = n1 - T(2.0 / 3.0) * m;
            n7 = n5 + T(0.5) * (n2 - n4) - m * T(1.0 / 6.0);
            n6 = n8 - T(0.5) * (n2 - n4) - m * T(1.0 / 6.0);
        }
    }
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
    s[4] = n4;
    s[5] = n5;
    s[6] = n6;
    s[7] = n7;
    s[8] = n8;
}

// Pulls the nine populations arriving at (x, y) from the post-collision field
// (pull_loads: the loads and the storage reference's row change) and completes
// the wall rows with Zou-He (unknowns from the knowns, tangential momentum
// target rho_w u_w - F_x / 2) and, in an open channel, the inlet and outlet
// columns (pull_complete).  OPEN = false compiles the periodic-x lattice only
// (the hot path, and callers that never reach the end columns of an open
// channel).  The split lets the grid pass issue the nine loads before it reads
// the segment's flags, whose value the completion (F_x) depends on.
template <typename T, bool OPEN = true>
__device__ __forceinline__ void pull_loads(const T* __restrict__ src, int x, int y,
                                           const GridArgs& g, T s[9])
{
    const size_t plane = (size_t)g.ny * g.nxp;
    int xm = x == 0 ? g.nx - 1 : x - 1;
    int xp = x == g.nx - 1 ? 0 : x + 1;
    if (OPEN && !g.periodic_x) {  // clamped: the unknown slots are replaced below
        xm = x == 0 ? 0 : xm;
        xp = x == g.nx - 1 ? x : xp;
    }
    int ym, yp;
    if (g.periodic_y) {
        ym = y == 0 ? g.ny - 1 : y - 1;
        yp = y == g.ny - 1 ? 0 : y + 1;
    } else {  // clamped: the out-of-domain slots are replaced by Zou-He below
        ym = y == 0 ? 0 : y - 1;
        yp = y == g.ny - 1 ? y : y + 1;
    }
    const size_t r0 = (size_t)y * g.nxp, rm = (size_t)ym * g.nxp, rp = (size_t)yp * g.nxp;
    s[0] = ld_stream(&src[r0 + x]);
    s[1] = src[plane + r0 + xm];
    s[2] = ld_stream(&src[2 * plane + rm + x]);
    s[3] = src[3 * plane + r0 + xp];
    s[4] = ld_stream(&src[4 * plane + rp + x]);
    s[5] = src[5 * plane + rm + xm];
    s[6] = src[6 * plane + rm + xp];
    s[7] = src[7 * plane + rp + xp];
    s[8] = src[8 * plane + rp + xm];
    add_pull_offsets(g, y, s);
}

template <typename T, bool OPEN = true>
__device__ __forceinline__ void pull_complete(const T* __restrict__ src, int x, int y,
                                              const GridArgs& g, T Fx, T s[9])
{
    if (OPEN && !g.periodic_x && (x == 0 || x == g.nx - 1)) {
        open_boundary(src, x, y, g, s);
        return;
    }
    if (!g.periodic_y && (y == 0 || y == g.ny - 1)) {
        // bottom row: s2, s5, s6 unknown from s4, s7, s8; top row: s4, s7, s8
        // from s2, s5, s6 (the same formulas with e_y and the sign of the
        // tangential terms mirrored).  Written with selects, so that every slot
        // of s stays a register.
        const bool top = y == g.ny - 1;
        const T a2 = top ? s[2] : s[4], a5 = top ? s[5] : s[7], a6 = top ? s[6] : s[8];
        const T rw = T(1) + s[0] + s[1] + s[3] + T(2) * (a2 + a5 + a6);
        const T mx = rw * (top ? (T)g.u_top : (T)g.u_bot) - T(0.5) * Fx;
        const T d13 = s[1] - s[3];
        const T h = top ? T(-0.5) : T(0.5);
        const T u5 = a5 - h * d13 + h * mx;  // bottom s5, top s7
        const T u6 = a6 + h * d13 - h * mx;  // bottom s6, top s8
        s[2] = top ? s[2] : a2;
        s[4] = top ? a2 : s[4];
        s[5] = top ? s[5] : u5;
        s[7] = top ? u5 : s[7];
        s[6] = top ? s[6] : u6;
        s[8] = top ? u6 : s[8];
    }
}

template <typename T, bool OPEN = true>
__device__ __forceinline__ void pull(const T* __restrict__ src, int x, int y, const GridArgs& g,
                                     T Fx, T s[9])
{
    pull_loads<T, OPEN>(src, x, y, g, s);
    pull_complete<T, OPEN>(src, x, y, g, Fx, s);
}

// Moments of the capsule's fluid patch, staged in LDS: density deviation
// rho - 1 and the force-corrected velocity.  Cells on a wall row hold NaN
// and raise ST_WALL if a support touches them.
template <typename T>
struct Patch {
    T* drho;
    T* ux;
    T* uy;
    int ox, oy, W, H;  // origin relative to the capsule reference point, size
};

template <typename T>
__device__ __forceinline__ bool patch_index(const Patch<T>& P, int cx, int cy, int k, int& idx)
{
    const int lx = cx + k % 3 - 1 - P.ox, ly = cy + k / 3 - 1 - P.oy;
    idx = ly * P.W + lx;
    return lx >= 0 && lx < P.W && ly >= 0 && ly < P.H;
}

// Moments of one patch cell from its pulled populations s (f^n) and the force
// F^{n-1} of the last collision (Eqs. 6-7, fixed-point force, g added):
// rho - 1 and the force-corrected velocity.
template <typename T>
__device__ __forceinline__ void stage_store(const Patch<T>& P, int i, const T (&s)[9],
                                            long long fx, long long fy, T gxf, T ur)
{
    const T Fx = gxf + fix_to_real<T>(fx);
    const T Fy = fix_to_real<T>(fy);
    const T drho = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])) + s[8];
    const T jx = (s[1] - s[3]) + (s[5] - s[6]) + (s[8] - s[7]);
    const T jy = (s[2] - s[4]) + (s[5] + s[6]) - (s[7] + s[8]);
    const T irho = T(1) / (T(1) + drho);
    P.drho[i] = drho;
    P.ux[i] = (ur + (jx + T(0.5) * Fx)) * irho;
    P.uy[i] = (jy + T(0.5) * Fy) * irho;
}

// Lattice coordinate ref + off on a periodic axis of n nodes.  The reference
// point (64-bit, unwrapped) is reduced once per call site with wrap_ref; each
// coordinate then takes an add and at most one correction while |off| < n, and
// the remainder only beyond that.  (A 64-bit remainder is a long software
// sequence on the GPU.)
__device__ __forceinline__ int wrap_ref(long long ref, int n)
{
    const long long r = ref % n;
    return (int)(r < 0 ? r + n : r);
}

__device__ __forceinline__ int wrap_add(int base, int off, int n)
{
    int v = base + off;
    if (v < 0) v += n;
    else if (v >= n) v -= n;
    if ((unsigned)v >= (unsigned)n) v = wrap_ref(v, n);
    return v;
}

// K patch cells first, first + stride, ..., with the loads of all of them
// issued before any is used (one memory latency for K cells).  A cell on a
// wall row or an open end column is marked NaN; cells past the patch store
// nothing (both load lattice cell (1, 1) instead).  A staged cell is never on
// a wall row or an end column, so its pull (the nine source addresses of the
// grid kernel's pull) needs no boundary rule.
template <typename T, int K>
__device__ __forceinline__ void stage_cells(const IBArgs<T>& a, const GridArgs& g,
                                            const Patch<T>& P, long long refx, long long refy,
                                            T gxf, int first, int stride)
{
    const int ncell = P.W * P.H;
    const size_t plane = (size_t)g.ny * g.nxp;
    const int bx = g.periodic_x ? wrap_ref(refx + P.ox, g.nx) : 0;
    const int by = g.periodic_y ? wrap_ref(refy + P.oy, g.ny) : 0;
    // patch column and row of cell `first`, advanced by `stride` per k
    int lx = first % P.W, ly = first / P.W;
    const int sx = stride % P.W, sy = stride / P.W;
    T s[K][9];
    long long fx[K], fy[K];
    int state[K];  // 0: past the patch, 1: off the lattice, 2: staged
    int row[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int i = first + k * stride;
        int x = 1, y = 1;
        state[k] = 0;
        if (i < ncell) {
            bool on = true;
            int wy, wx;
            if (g.periodic_y) {
                wy = wrap_add(by, ly, g.ny);
            } else {
                const long long v = refy + P.oy + ly;
                on = v >= 1 && v <= g.ny - 2;
                wy = (int)v;
            }
            if (g.periodic_x) {
                wx = wrap_add(bx, lx, g.nx);
            } else {
                const long long v = refx + P.ox + lx;
                on = on && v >= 1 && v <= g.nx - 2;
                wx = (int)v;
            }
            state[k] = on ? 2 : 1;
            if (on) {
                x = wx;
                y = wy;
            }
        }
        lx += sx;
        ly += sy;
        if (lx >= P.W) {
            lx -= P.W;
            ly++;
        }
        const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        const size_t r0 = (size_t)y * g.nxp, rm = (size_t)ym * g.nxp, rp = (size_t)yp * g.nxp;
        const T* src = a.pops;
        s[k][0] = src[r0 + x];
        s[k][1] = src[plane + r0 + xm];
        s[k][2] = src[2 * plane + rm + x];
        s[k][3] = src[3 * plane + r0 + xp];
        s[k][4] = src[4 * plane + rp + x];
        s[k][5] = src[5 * plane + rm + xm];
        s[k][6] = src[6 * plane + rm + xp];
        s[k][7] = src[7 * plane + rp + xp];
        s[k][8] = src[8 * plane + rp + xm];
        row[k] = y;
        const longlong2 f = *reinterpret_cast<const longlong2*>(a.fib_prev + 2 * (r0 + x));
        fx[k] = f.x;
        fy[k] = f.y;
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int i = first + k * stride;
        if (state[k] == 2) {
            add_pull_offsets(g, row[k], s[k]);
            stage_store(P, i, s[k], fx[k], fy[k], gxf, uref_at<T>(g, row[k]));
        } else if (state[k] == 1) {
            P.drho[i] = T(NAN);
            P.ux[i] = P.uy[i] = T(0);
        }
    }
}

// Wave-wide reductions with DPP lane moves (register to register, no LDS
// round trip): exchange within lane pairs and quads (quad_perm), mirror within
// half-rows and rows of 16, then the row broadcasts of lanes 15 and 31 carry
// the row results into the last row.  Lane 63 ends with the result, which is
// broadcast from there; the combination order is fixed by the lane pattern.
// Call with the whole wave active.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move_f64(double v)  // rows outside ROWS read 0
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_move<CTRL, ROWS>(0, (int)(unsigned int)(b & 0xffffffffLL));
    const int hi = dpp_move<CTRL, ROWS>(0, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move_f64<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move_f64<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_move_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_move_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move_f32(float v)  // rows outside ROWS keep v
{
    return __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(v), __float_as_int(v)));
}

template <bool MAX>
__device__ __forceinline__ float wave_extreme(float v)
{
#define LBIB_STEP(C, R)                         \
    {                                           \
        const float o = dpp_move_f32<C, R>(v);  \
        v = MAX ? fmaxf(v, o) : fminf(v, o);    \
    }
    LBIB_STEP(0xB1, 0xF)
    LBIB_STEP(0x4E, 0xF)
    LBIB_STEP(0x141, 0xF)
    LBIB_STEP(0x140, 0xF)
    LBIB_STEP(0x142, 0xA)
    LBIB_STEP(0x143, 0xC)
#undef LBIB_STEP
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Deterministic block reductions over the wavefronts of a block (at most
// kIBThreads / 64): a DPP reduction within each wave, then the wave partials in
// order.

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*red)[8])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; k++) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; k++) red[wave][k] = v[k];
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
#pragma unroll
    for (int k = 0; k < N; k++) {
        double acc = red[0][k];
        for (int w = 1; w < nw; w++) acc += red[w][k];
        v[k] = acc;
    }
    __syncthreads();
}

__device__ __forceinline__ void block_minmax(float (&mn)[2], float (&mx)[2], double (*red)[8],
                                             bool closing_barrier = true)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 2; k++) {
        mn[k] = wave_extreme<false>(mn[k]);
        mx[k] = wave_extreme<true>(mx[k]);
    }
    if (lane == 0) {
        red[wave][0] = mn[0];
        red[wave][1] = mn[1];
        red[wave][2] = mx[0];
        red[wave][3] = mx[1];
    }
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    for (int k = 0; k < 2; k++) {
        float a = (float)red[0][k], b = (float)red[0][2 + k];
        for (int w = 1; w < nw; w++) {
            a = fminf(a, (float)red[w][k]);
            b = fmaxf(b, (float)red[w][2 + k]);
        }
        mn[k] = a;
        mx[k] = b;
    }
    if (closing_barrier) __syncthreads();
}

}  // namespace lbib
