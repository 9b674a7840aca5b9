// Reverse-mode (adjoint) kernels of the LBM - immersed boundary step
// (arXiv:1903.03356, Secs. 2.1-2.4): gradients of an objective of the final
// capsule shape (Taylor deformation or area-centroid height, Sec. 3) with
// respect to the per-element stretching constants k_s (Eq. 10) and the
// uniform body force g that drives the channel.
//
// The forward run is taped in full (populations, IB force field and node
// state of every time level), so the reverse sweep recomputes nothing.  Each
// reverse time step is one grid kernel (transpose of collide + stream + walls)
// and one IB kernel (transpose of the Lagrangian update and of the forcing).
// Derivatives of the MLS shape functions (Eq. 9) with respect to the marker or
// probe position are carried by forward-mode dual numbers, so every local
// Jacobian is exact; the transposed products are assembled by hand.
//
// Scope: both coupling schemes, membranes with stretching, bending and area
// terms, one lattice per context.  The support of every MLS stencil is the one the
// forward run chose (piecewise constant in the position, so its derivative is
// zero).
#include "lbib_adjoint.h"
#include "lbib_device.h"

namespace lbib {

// The reverse IB kernel runs 256 threads per capsule: one wave per SIMD, so
// its dual-number MLS work gets the whole register file instead of spilling.
constexpr int kAdjThreads = 256;

// ------------------------------------------------------------ dual numbers
template <int N>
struct Dual {
    double v;
    double d[N];
};

template <int N>
__device__ __forceinline__ Dual<N> dconst(double c)
{
    Dual<N> r;
    r.v = c;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = 0.0;
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> dvar(double c, int k)
{
    Dual<N> r = dconst<N>(c);
    r.d[k] = 1.0;
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = a.d[i] + b.d[i];
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = a.d[i] - b.d[i];
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator*(double s, const Dual<N>& a)
{
    Dual<N> r;
    r.v = s * a.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = s * a.d[i];
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double s)
{
    Dual<N> r = a;
    r.v += s;
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> dinv(const Dual<N>& a)
{
    const double iv = 1.0 / a.v;
    Dual<N> r;
    r.v = iv;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = -a.d[i] * iv * iv;
    return r;
}

template <int N>
__device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a)
{
    const double s = sqrt(a.v);
    Dual<N> r;
    r.v = s;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = a.d[i] * 0.5 / s;
    return r;
}

// ----------------------------------------------------------- MLS with slopes
// Shape functions of Eq. 9 at p = (px, py) (FP64, patch frame) on the 3x3
// support centred at (cx, cy), together with their partial derivatives with
// respect to p.  Weight, basis and moment matrix follow the forward kernel
// (marker-centred linear basis, W = exp(-(r / (2.6 * 0.3))^2)).  For every
// support node k, f(k, phi, gx, gy) receives the value row and, if G, the two
// slope rows (diffuse derivatives), each as a dual over (px, py).
template <bool G, typename F>
__device__ __forceinline__ void mls_dual(double px, double py, int cx, int cy, F&& f)
{
    using D = Dual<2>;
    const double inv2 = 1.0 / (2.6 * 0.3 * 2.6 * 0.3);
    D a00 = dconst<2>(0), a01 = a00, a02 = a00, a11 = a00, a12 = a00, a22 = a00;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const double X = (double)(cx + k % 3 - 1) - px, Y = (double)(cy + k / 3 - 1) - py;
        const double e = exp(-(X * X + Y * Y) * inv2);
        D w;
        w.v = e;
        w.d[0] = 2.0 * X * inv2 * e;  // dX/dpx = -1
        w.d[1] = 2.0 * Y * inv2 * e;
        D Xd, Yd;
        Xd.v = X;
        Xd.d[0] = -1.0;
        Xd.d[1] = 0.0;
        Yd.v = Y;
        Yd.d[0] = 0.0;
        Yd.d[1] = -1.0;
        const D wX = w * Xd, wY = w * Yd;
        a00 = a00 + w;
        a01 = a01 + wX;
        a02 = a02 + wY;
        a11 = a11 + wX * Xd;
        a12 = a12 + wX * Yd;
        a22 = a22 + wY * Yd;
    }
    const D c00 = a11 * a22 - a12 * a12;
    const D c01 = a02 * a12 - a01 * a22;
    const D c02 = a01 * a12 - a02 * a11;
    const D id = dinv(a00 * c00 + a01 * c01 + a02 * c02);
    const D i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    D i11 = dconst<2>(0), i12 = i11, i22 = i11;
    if (G) {
        i11 = (a00 * a22 - a02 * a02) * id;
        i12 = (a01 * a02 - a00 * a12) * id;
        i22 = (a00 * a11 - a01 * a01) * id;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const double X = (double)(cx + k % 3 - 1) - px, Y = (double)(cy + k / 3 - 1) - py;
        const double e = exp(-(X * X + Y * Y) * inv2);
        D w;
        w.v = e;
        w.d[0] = 2.0 * X * inv2 * e;
        w.d[1] = 2.0 * Y * inv2 * e;
        D Xd, Yd;
        Xd.v = X;
        Xd.d[0] = -1.0;
        Xd.d[1] = 0.0;
        Yd.v = Y;
        Yd.d[0] = 0.0;
        Yd.d[1] = -1.0;
        const D phi = w * (i00 + i01 * Xd + i02 * Yd);
        D gx = dconst<2>(0), gy = gx;
        if (G) {
            gx = w * (i01 + i11 * Xd + i12 * Yd);
            gy = w * (i02 + i12 * Xd + i22 * Yd);
        }
        f(k, phi, gx, gy);
    }
}

// ---------------------------------------------------------- grid reverse
// Transpose of one grid step at one node.  The forward map is
//   out = C(ZH(pull(P^n), F), F),  F = g + f_ib^n at the node,
// with C the BGK + forcing relaxation of the deviations (Eqs. 2, 4-7) and ZH
// the Zou-He completion of a wall row.  Given lambda of out (the adjoint of
// P^{n+1} at this node), it returns the adjoint of the nine pulled values and
// of F.
template <typename T>
__device__ __forceinline__ void collide_vjp(const T s[9], T Fx, T Fy, T ur, T om, const T lo[9],
                                            T sb[9], T& Fbx, T& Fby)
{
    const T drho = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])) + s[8];
    const T rho = T(1) + drho;
    const T jx = (s[1] - s[3]) + (s[5] - s[6]) + (s[8] - s[7]);
    const T jy = (s[2] - s[4]) + (s[5] + s[6]) - (s[7] + s[8]);
    const T irho = T(1) / rho;
    const T mx = jx + T(0.5) * Fx, my = jy + T(0.5) * Fy;
    const T ux = (ur + mx) * irho, uy = my * irho;  // ur: storage reference u_ref(y)
    const T pre = T(1) - T(0.5) * om;
    const T usq15 = T(1.5) * (ux * ux + uy * uy);
    T drhob = 0, rhob = 0, mbx = 0, mby = 0, ubx = 0, uby = 0, usqb = 0, uFb = 0;
    Fbx = Fby = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const T w = lat_w<T>(i);
        const T w3 = i == 0 ? T(0) : (i < 5 ? FirstOrderW<T>::axis : FirstOrderW<T>::diag);
        const T ex = (T)kEx[i], ey = (T)kEy[i];
        const T eu = ex * ux + ey * uy;
        const T eF = ex * Fx + ey * Fy;
        const T q = om * lo[i];  // adjoint of the equilibrium term
        const T r = lo[i];       // adjoint of the forcing term
        sb[i] = (T(1) - om) * lo[i];
        drhob += w * q;
        mbx += w3 * q * ex;
        mby += w3 * q * ey;
        rhob += w * q * (T(4.5) * eu * eu - usq15);
        const T cu = T(9) * w * (rho * eu * q + pre * eF * r);
        ubx += cu * ex;
        uby += cu * ey;
        usqb -= w * rho * q;
        const T cF = pre * (w3 + T(9) * w * eu) * r;
        Fbx += cF * ex;
        Fby += cF * ey;
        uFb -= T(3) * pre * w * r;
    }
    ubx += T(3) * ux * usqb + Fx * uFb;
    uby += T(3) * uy * usqb + Fy * uFb;
    Fbx += ux * uFb;
    Fby += uy * uFb;
    mbx += ubx * irho;
    mby += uby * irho;
    rhob -= (ux * ubx + uy * uby) * irho;
    Fbx += T(0.5) * mbx;
    Fby += T(0.5) * mby;
    drhob += rhob;
#pragma unroll
    for (int i = 0; i < 9; i++) sb[i] += drhob + (T)kEx[i] * mbx + (T)kEy[i] * mby;
}

// Transpose of the Zou-He completion of the bottom (top = false) or top wall
// row: folds the adjoint of the three unknowns onto the six pulled knowns and
// the x-force.  The unknown slots' own pulled values are discarded, so their
// adjoint becomes zero.
template <typename T>
__device__ __forceinline__ void zou_he_vjp(T sb[9], T& Fbx, T uw, bool top)
{
    if (!top) {
        const T lm = T(0.5) * (sb[5] - sb[6]);  // adjoint of rho_w u_w - F_x / 2
        const T c = lm * uw;
        sb[0] += c;
        sb[1] += c - T(0.5) * sb[5] + T(0.5) * sb[6];
        sb[3] += c + T(0.5) * sb[5] - T(0.5) * sb[6];
        sb[4] += sb[2] + T(2) * c;
        sb[7] += sb[5] + T(2) * c;
        sb[8] += sb[6] + T(2) * c;
        sb[2] = sb[5] = sb[6] = T(0);
        Fbx -= T(0.5) * lm;
    } else {
        const T lm = T(0.5) * (sb[8] - sb[7]);
        const T c = lm * uw;
        sb[0] += c;
        sb[1] += c + T(0.5) * sb[7] - T(0.5) * sb[8];
        sb[3] += c - T(0.5) * sb[7] + T(0.5) * sb[8];
        sb[2] += sb[4] + T(2) * c;
        sb[5] += sb[7] + T(2) * c;
        sb[6] += sb[8] + T(2) * c;
        sb[4] = sb[7] = sb[8] = T(0);
        Fbx -= T(0.5) * lm;
    }
}

__device__ __forceinline__ void block_add_partial(double v, double* slot)
{
    __shared__ double part[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) *slot += ((part[0] + part[1]) + (part[2] + part[3]));
}

// One reverse grid step.  Same block-to-cell mapping as the forward grid
// kernel.  Writes lambda P^n (every slot of every node, pushed to where the
// forward pull read it), lambda F^n at the active force segments, and adds
// sum_x lambda F_x (the body-force gradient of this step) to the block's slot.
template <typename T>
__global__ __launch_bounds__(kSegW * 4) void k_grid_adj(GridAdjArgs<T> a, GridArgs g)
{
    const int b = blockIdx.x;
    const int j = b / kNumXcd;
    const int group = j / g.nseg;
    const int band = group * kNumXcd + (b - j * kNumXcd);
    const int seg = j - group * g.nseg;
    const int lane = threadIdx.x & (kSegW - 1);
    const int y = band * 4 + (threadIdx.x >> 6);
    double gsum = 0.0;
    if (y < g.ny) {
        const int x = seg * kSegW + lane;
        const int fidx = y * g.nseg + seg;
        const int act = a.flags[fidx];
        const int mflag = a.lfm_flags[fidx];
        const size_t cell = (size_t)y * g.nxp + x;
        const size_t plane = (size_t)g.ny * g.nxp;
        if (x < g.nx) {
            T Fx = (T)g.gx, Fy = T(0);
            if (act) {
                Fx += fix_to_real<T>(a.fib[2 * cell]);
                Fy += fix_to_real<T>(a.fib[2 * cell + 1]);
            }
            T s[9], lo[9], sb[9];
            pull<T, false>(a.pops, x, y, g, Fx, s);  // the adjoint needs periodic x
#pragma unroll
            for (int i = 0; i < 9; i++) lo[i] = a.lam_in[i * plane + cell];
            T Fbx, Fby;
            collide_vjp(s, Fx, Fy, uref_at<T>(g, y), (T)g.omega, lo, sb, Fbx, Fby);
            const bool bot = !g.periodic_y && y == 0, top = !g.periodic_y && y == g.ny - 1;
            if (bot) zou_he_vjp(sb, Fbx, (T)g.u_bot, false);
            if (top) zou_he_vjp(sb, Fbx, (T)g.u_top, true);
            if (mflag) {
                Fbx += a.lfm[2 * cell];
                Fby += a.lfm[2 * cell + 1];
            }
            gsum = (double)Fbx;
            if (act) {
                a.lft[2 * cell] = Fbx;
                a.lft[2 * cell + 1] = Fby;
            }
            const int xm = x == 0 ? g.nx - 1 : x - 1;
            const int xp = x == g.nx - 1 ? 0 : x + 1;
#pragma unroll
            for (int i = 0; i < 9; i++) {
                int xs = kEx[i] > 0 ? xm : (kEx[i] < 0 ? xp : x);
                int ys = y - kEy[i];
                if (g.periodic_y) ys = ys < 0 ? g.ny - 1 : (ys >= g.ny ? 0 : ys);
                else if (ys < 0 || ys >= g.ny) continue;
                a.lam_out[i * plane + (size_t)ys * g.nxp + xs] = sb[i];
            }
            // slots that no node pulls from (they point out of the walls)
            if (bot) {
                a.lam_out[4 * plane + cell] = T(0);
                a.lam_out[7 * plane + cell] = T(0);
                a.lam_out[8 * plane + cell] = T(0);
            }
            if (top) {
                a.lam_out[2 * plane + cell] = T(0);
                a.lam_out[5 * plane + cell] = T(0);
                a.lam_out[6 * plane + cell] = T(0);
            }
        }
        if (mflag) {
            a.lfm[2 * cell] = T(0);
            a.lfm[2 * cell + 1] = T(0);
            if (lane == 0) a.lfm_flags[fidx] = 0;
        }
    }
    block_add_partial(gsum, a.gacc + b);
}

// Initial state: P^0 = f_eq(1, u_0(y)) - w (Eq. 2) with the body-force
// Poiseuille profile u_0 = g / (2 nu) y (H - y) depends on g; the moments of
// the first step also used F^{-1} = g.  Adds both terms to the block slots.
template <typename T>
__global__ __launch_bounds__(kSegW * 4) void k_init_adj(GridAdjArgs<T> a, GridArgs g,
                                                       int profile, double nu)
{
    const int b = blockIdx.x;
    const int j = b / kNumXcd;
    const int group = j / g.nseg;
    const int band = group * kNumXcd + (b - j * kNumXcd);
    const int seg = j - group * g.nseg;
    const int lane = threadIdx.x & (kSegW - 1);
    const int y = band * 4 + (threadIdx.x >> 6);
    double gsum = 0.0;
    if (y < g.ny) {
        const int x = seg * kSegW + lane;
        const size_t cell = (size_t)y * g.nxp + x;
        const size_t plane = (size_t)g.ny * g.nxp;
        if (x < g.nx) {
            if (profile == 2) {
                const double H = g.ny - 1;
                for (int i = 0; i < 9; i++) {
                    int yd = y + kEy[i];
                    if (g.periodic_y) yd = (yd + g.ny) % g.ny;
                    else yd = yd < 0 ? 0 : (yd > g.ny - 1 ? g.ny - 1 : yd);
                    const double ux = g.gx / (2.0 * nu) * yd * (H - yd);
                    const double dux = yd * (H - yd) / (2.0 * nu);
                    const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
                    const double ex = kEx[i];
                    gsum += (double)a.lam_in[i * plane + cell] * w *
                            (3.0 * ex + 9.0 * ex * ex * ux - 3.0 * ux) * dux;
                }
            }
            if (a.lfm_flags[y * g.nseg + seg]) gsum += (double)a.lfm[2 * cell];
        }
    }
    block_add_partial(gsum, a.gacc + b);
}

__global__ void k_reduce_sum(const double* v, int n, double* out)
{
    __shared__ double part[kIBThreads / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += part[w];
        *out = t;
    }
}

// ------------------------------------------------------------ objective
// Polygon sums of Green's theorem over element (x0, y0) -> (x1, y1):
// 2A, x and y first moments (times 6), second moments (times 12, 12, 24).
template <int N>
__device__ __forceinline__ void element_sums(const Dual<N>& x0, const Dual<N>& y0,
                                             const Dual<N>& x1, const Dual<N>& y1, Dual<N> (&S)[6])
{
    const Dual<N> cr = x0 * y1 - x1 * y0;
    S[0] = cr;
    S[1] = (x0 + x1) * cr;
    S[2] = (y0 + y1) * cr;
    S[3] = (x0 * x0 + x0 * x1 + x1 * x1) * cr;
    S[4] = (y0 * y0 + y0 * y1 + y1 * y1) * cr;
    S[5] = (x0 * y1 + 2.0 * (x0 * y0) + 2.0 * (x1 * y1) + x1 * y0) * cr;
}

// Objective from the six sums (same formulas as the diagnostics): Taylor
// deformation of the equivalent ellipse (objective 0) or the area-centroid
// height relative to the reference point (objective 1).
template <int N>
__device__ __forceinline__ Dual<N> objective_of(const Dual<N> (&S)[6], int objective)
{
    const Dual<N> A = 0.5 * S[0];
    const Dual<N> iA6 = dinv(3.0 * S[0]);  // 1 / (6 A)
    const Dual<N> cx = S[1] * iA6, cy = S[2] * iA6;
    if (objective == 1) return cy;
    const Dual<N> jxx = (1.0 / 12.0) * S[3] - A * cx * cx;
    const Dual<N> jyy = (1.0 / 12.0) * S[4] - A * cy * cy;
    const Dual<N> jxy = (1.0 / 24.0) * S[5] - A * cx * cy;
    const Dual<N> tr = 0.5 * (jxx + jyy);
    const Dual<N> dd = jxx - jyy;
    const Dual<N> disc = dsqrt(0.25 * (dd * dd) + jxy * jxy);
    const Dual<N> sa = dsqrt(tr + disc), sb = dsqrt(tr - disc);
    return (sa - sb) * dinv(sa + sb);
}

// One block: J of capsule `cap_id` from the node positions of the final tape
// slot, and its gradient with respect to every node coordinate (the seed of
// the reverse sweep).  out[1] = J.
template <typename T>
__global__ __launch_bounds__(kIBThreads) void k_adj_seed(const T* nodes, const double* ref,
                                                        const CapsuleDev* caps, int cap_id,
                                                        int stride, int objective, double* lamx,
                                                        double* out)
{
    __shared__ double red[kIBThreads / 64][8];
    const CapsuleDev cap = caps[cap_id];
    const int nv = cap.nv, off = cap.node_offset;
    const size_t NS = stride;
    auto X = [&](int v) {
        return (double)nodes[NF_HX * NS + off + v] + (double)nodes[NF_LX * NS + off + v];
    };
    auto Y = [&](int v) {
        return (double)nodes[NF_HY * NS + off + v] + (double)nodes[NF_LY * NS + off + v];
    };
    double sums[6] = {0, 0, 0, 0, 0, 0};
    for (int l = threadIdx.x; l < nv; l += blockDim.x) {
        const int m = l + 1 == nv ? 0 : l + 1;
        Dual<4> S[6];
        element_sums<4>(dconst<4>(X(l)), dconst<4>(Y(l)), dconst<4>(X(m)), dconst<4>(Y(m)), S);
        for (int k = 0; k < 6; k++) sums[k] += S[k].v;
    }
    block_sum<6>(sums, red);
    Dual<6> Sd[6];
    for (int k = 0; k < 6; k++) Sd[k] = dvar<6>(sums[k], k);
    const Dual<6> J = objective_of<6>(Sd, objective);
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
        Dual<4> Sa[6], Sb[6];
        // element vl -> v: node v is the end point (partials 2, 3)
        element_sums<4>(dconst<4>(X(vl)), dconst<4>(Y(vl)), dvar<4>(X(v), 2), dvar<4>(Y(v), 3), Sa);
        // element v -> vr: node v is the start point (partials 0, 1)
        element_sums<4>(dvar<4>(X(v), 0), dvar<4>(Y(v), 1), dconst<4>(X(vr)), dconst<4>(Y(vr)), Sb);
        double gx = 0, gy = 0;
        for (int k = 0; k < 6; k++) {
            gx += J.d[k] * (Sa[k].d[2] + Sb[k].d[0]);
            gy += J.d[k] * (Sa[k].d[3] + Sb[k].d[1]);
        }
        lamx[off + v] = gx;
        lamx[NS + off + v] = gy;
    }
    if (threadIdx.x == 0) out[1] = J.v + (objective == 1 ? ref[2 * cap_id + 1] : 0.0);
}

// --------------------------------------------------------------- IB reverse
// LDS layout of the IB reverse kernel: the staged moments M^n of the patch and
// their adjoints (T), the node coordinates the forward kernel used to choose
// MLS supports (T), and per-node FP64 work arrays.
template <typename T>
struct AdjScratch {
    T *pd, *pu, *pv;  // staged rho - 1, ux, uy
    T *Ld, *Lu, *Lv;  // their adjoints
    T *hxn, *hyn;     // x^n high parts (frame n)
    T *hxp, *hyp, *lxp, *lyp;  // x^{n-1} high and low parts (frame n-1)
    double *Xn, *Yn, *Xp, *Yp;  // positions in the patch frame (FP64)
    double *uvx, *uvy;          // u_v^n
    double *lx, *ly;            // lambda x (carried)
    double *ldx, *ldy;          // lambda d (carried)
    double *lux, *luy;          // lambda u_v^n
    double *lFx, *lFy;          // lambda of the nodal force
    double *lc;                 // lambda c_v
    double *E1x, *E1y, *E2x, *E2y;  // element contributions to its start / end node
    double *Fvx, *Fvy;          // forward nodal force (Kinematic forcing)
};

constexpr int kAdjDoubleArrays = 21;
constexpr int kAdjRealNodeArrays = 6;
constexpr int kAdjRealCellArrays = 6;

template <typename T>
size_t ib_adj_lds_bytes(int patch_cap, int max_nv)
{
    size_t b = sizeof(T) * ((size_t)kAdjRealCellArrays * patch_cap +
                            (size_t)kAdjRealNodeArrays * max_nv);
    b = (b + 15) & ~(size_t)15;
    return b + sizeof(double) * (size_t)kAdjDoubleArrays * max_nv;
}

// Patch index of support node k of the stencil centred at (cx, cy) (patch
// frame); -1 if outside the staged patch or on a wall row.
template <typename T>
__device__ __forceinline__ int adj_patch_index(const Patch<T>& P, int cx, int cy, int k)
{
    const int lx = cx + k % 3 - 1 - P.ox, ly = cy + k / 3 - 1 - P.oy;
    if (lx < 0 || lx >= P.W || ly < 0 || ly >= P.H) return -1;
    const int idx = ly * P.W + lx;
    return isnan(P.drho[idx]) ? -1 : idx;
}

// Transpose of the interpolation v = sum_k phi_k(p) u_k (Eq. 8) for a given
// adjoint lv of v: adds phi_k lv to the velocity adjoints of the support and
// returns d(lv . v)/dp.
template <typename T>
__device__ __forceinline__ void interp_vjp(const AdjScratch<T>& S, const Patch<T>& P, double px,
                                           double py, int cx, int cy, double lvx, double lvy,
                                           double& gpx, double& gpy, int& st)
{
    gpx = gpy = 0.0;
    mls_dual<false>(px, py, cx, cy, [&](int k, const Dual<2>& phi, const Dual<2>&, const Dual<2>&) {
        const int idx = adj_patch_index(P, cx, cy, k);
        if (idx < 0) { st |= ST_PATCH; return; }
        const double u = (double)S.pu[idx], v = (double)S.pv[idx];
        const double c = u * lvx + v * lvy;
        gpx += c * phi.d[0];
        gpy += c * phi.d[1];
        atomicAdd(&S.Lu[idx], (T)(phi.v * lvx));
        atomicAdd(&S.Lv[idx], (T)(phi.v * lvy));
    });
}

// Bending at vertex v (Eq. 13: the outer terms as printed, the middle node
// minus their sum, which is minus the gradient of k_b (1 - cos(theta - theta0))).
// Left edge a = x_v - x_{v-1}, right edge b = x_{v+1} - x_v, theta the signed
// turning angle.  The left neighbour takes s P(a), the right one s P(b) and
// the vertex minus both, with s = k_b sin(theta - theta0) and
// P(t) = (t_y, -t_x) / |t|^2.
struct BendAt {
    double s, c;        // k_b sin(theta - theta0), k_b cos(theta - theta0)
    double ax, ay, na;  // left edge and its squared length
    double bx, by, nb;  // right edge and its squared length
};

__device__ __forceinline__ BendAt bend_at(const double* X, const double* Y, int v, int nv,
                                          double kb, double th0)
{
    const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
    BendAt r;
    r.ax = X[v] - X[vl];
    r.ay = Y[v] - Y[vl];
    r.bx = X[vr] - X[v];
    r.by = Y[vr] - Y[v];
    r.na = r.ax * r.ax + r.ay * r.ay;
    r.nb = r.bx * r.bx + r.by * r.by;
    const double th = atan2(r.ax * r.by - r.ay * r.bx, r.ax * r.bx + r.ay * r.by);
    r.s = kb * sin(th - th0);
    r.c = kb * cos(th - th0);
    return r;
}

// Bending force on node v: the right-neighbour term of vertex v - 1, the
// left-neighbour term of vertex v + 1 and minus both terms of vertex v.
template <typename T>
__device__ __forceinline__ void bend_node_force(const double* X, const double* Y, int v, int nv,
                                                double kb, const T* th0, double& fx, double& fy)
{
    const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
    const BendAt L = bend_at(X, Y, vl, nv, kb, (double)th0[vl]);
    const BendAt M = bend_at(X, Y, v, nv, kb, (double)th0[v]);
    const BendAt R = bend_at(X, Y, vr, nv, kb, (double)th0[vr]);
    fx = L.s * L.by / L.nb + R.s * R.ay / R.na - M.s * (M.ay / M.na + M.by / M.nb);
    fy = -L.s * L.bx / L.nb - R.s * R.ax / R.na + M.s * (M.ax / M.na + M.bx / M.nb);
}

// Adjoint of edge l -> l+1 from the bending terms, for the nodal adjoint
// (lFx, lFy): the edge is the right edge b of vertex l and the left edge a of
// vertex l + 1.  Per vertex, g = s (hL . P(a) + hR . P(b)) with hL, hR the
// differences of the neighbours' adjoints from the vertex's; with
// Q = hL . P(a) + hR . P(b), dtheta/da = P(a) and dtheta/db = -P(b):
//   dg/da =  c Q P(a) + s ((-hL_y, hL_x) - 2 (hL . P(a)) a) / |a|^2,
//   dg/db = -c Q P(b) + s ((-hR_y, hR_x) - 2 (hR . P(b)) b) / |b|^2.
template <typename T>
__device__ __forceinline__ void bend_edge_vjp(const AdjScratch<T>& S, const double* X,
                                              const double* Y, int l, int nv, double kb,
                                              const T* th0, double& ltx, double& lty)
{
    const int m = l + 1 == nv ? 0 : l + 1;
    {   // vertex l, right edge
        const int vl = l == 0 ? nv - 1 : l - 1;
        const BendAt V = bend_at(X, Y, l, nv, kb, (double)th0[l]);
        const double hLx = S.lFx[vl] - S.lFx[l], hLy = S.lFy[vl] - S.lFy[l];
        const double hRx = S.lFx[m] - S.lFx[l], hRy = S.lFy[m] - S.lFy[l];
        const double qL = (hLx * V.ay - hLy * V.ax) / V.na;
        const double qR = (hRx * V.by - hRy * V.bx) / V.nb;
        const double cQ = V.c * (qL + qR);
        ltx += (-cQ * V.by + V.s * (-hRy - 2.0 * qR * V.bx)) / V.nb;
        lty += (cQ * V.bx + V.s * (hRx - 2.0 * qR * V.by)) / V.nb;
    }
    {   // vertex l + 1, left edge
        const int mr = m + 1 == nv ? 0 : m + 1;
        const BendAt W = bend_at(X, Y, m, nv, kb, (double)th0[m]);
        const double hLx = S.lFx[l] - S.lFx[m], hLy = S.lFy[l] - S.lFy[m];
        const double hRx = S.lFx[mr] - S.lFx[m], hRy = S.lFy[mr] - S.lFy[m];
        const double qL = (hLx * W.ay - hLy * W.ax) / W.na;
        const double qR = (hRx * W.by - hRy * W.bx) / W.nb;
        const double cQ = W.c * (qL + qR);
        ltx += (cQ * W.ay + W.s * (-hLy - 2.0 * qL * W.ax)) / W.na;
        lty += (-cQ * W.ax + W.s * (hLx - 2.0 * qL * W.ay)) / W.na;
    }
}

// Transpose of the internal forces (Eqs. 10-11 stretch, Eq. 13 bending, Eq.
// 14 area) at positions (X, Y) for the nodal adjoint (lFx, lFy): element
// contributions into E1 (start node) / E2 (end node), k_s gradient into
// ksbar, and the area term straight into the returned lambda A.
template <bool BEND, typename T>
__device__ double internal_vjp(const AdjScratch<T>& S, const double* X, const double* Y, int nv,
                               const T* l0h, const T* l0l, const T* ks, double kb, const T* th0,
                               double ka, double A0, double* ksbar, double (*red)[8])
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double acc[1] = {0.0};
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        acc[0] += X[l] * Y[m] - X[m] * Y[l];
    }
    block_sum<1>(acc, red);
    const double A = 0.5 * acc[0];
    const double cA = 0.5 * ka * (1.0 - A / A0) / 3.0;
    double lcA[1] = {0.0};
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        const double tx = X[m] - X[l], ty = Y[m] - Y[l];
        const double len = sqrt(tx * tx + ty * ty);
        const double L0 = (double)l0h[l] + (double)l0l[l];
        const double k = (double)ks[l];
        const double hSx = S.lFx[l] - S.lFx[m], hSy = S.lFy[l] - S.lFy[m];
        const double hAx = S.lFx[l] + S.lFx[m], hAy = S.lFy[l] + S.lFy[m];
        const double th = tx * hSx + ty * hSy;
        const double kap = k * (1.0 - L0 / len);
        const double q = k * L0 / (len * len * len) * th;
        // stretch: s = k (1 - l0/len) t
        double ltx = kap * hSx + q * tx, lty = kap * hSy + q * ty;
        ksbar[l] += (1.0 - L0 / len) * th;
        // area: a = cA (t_y, -t_x)
        ltx += -cA * hAy;
        lty += cA * hAx;
        lcA[0] += ty * hAx - tx * hAy;
        if (BEND && kb != 0.0) bend_edge_vjp(S, X, Y, l, nv, kb, th0, ltx, lty);
        S.E1x[l] -= ltx;
        S.E1y[l] -= lty;
        S.E2x[l] += ltx;
        S.E2y[l] += lty;
    }
    block_sum<1>(lcA, red);
    return -ka / (6.0 * A0) * lcA[0];
}

// Forward internal forces at (X, Y) (FP64) into (Fvx, Fvy): stretch, bending
// and area.
template <bool BEND, typename T>
__device__ void internal_fwd(const AdjScratch<T>& S, const double* X, const double* Y, int nv,
                             const T* l0h, const T* l0l, const T* ks, double kb, const T* th0,
                             double ka, double A0, double (*red)[8])
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double acc[1] = {0.0};
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        acc[0] += X[l] * Y[m] - X[m] * Y[l];
    }
    block_sum<1>(acc, red);
    const double cA = 0.5 * ka * (1.0 - 0.5 * acc[0] / A0) / 3.0;
    for (int l = tid; l < nv; l += nt) {
        const int m = l + 1 == nv ? 0 : l + 1;
        const double tx = X[m] - X[l], ty = Y[m] - Y[l];
        const double len = sqrt(tx * tx + ty * ty);
        const double L0 = (double)l0h[l] + (double)l0l[l];
        const double c = (double)ks[l] * (1.0 - L0 / len);
        S.E1x[l] = c * tx + cA * ty;  // onto node l
        S.E1y[l] = c * ty - cA * tx;
        S.E2x[l] = -c * tx + cA * ty;  // onto node l + 1
        S.E2y[l] = -c * ty - cA * tx;
    }
    __syncthreads();
    for (int v = tid; v < nv; v += nt) {
        const int vl = v == 0 ? nv - 1 : v - 1;
        double bx = 0.0, by = 0.0;
        if (BEND && kb != 0.0) bend_node_force(X, Y, v, nv, kb, th0, bx, by);
        S.Fvx[v] = S.E1x[v] + S.E2x[vl] + bx;
        S.Fvy[v] = S.E1y[v] + S.E2y[vl] + by;
    }
    __syncthreads();
    for (int l = tid; l < nv; l += nt) S.E1x[l] = S.E1y[l] = S.E2x[l] = S.E2y[l] = 0.0;
    __syncthreads();
}

// Transpose of the hydrodynamic forces (Eqs. 15-16) at x^{n-1}: element l
// force f = len (-(p+ - p-) n + (tau+ - tau-) n) split half and half, probes
// x_c +- 1.2 n.  hE = (lF_l + lF_m) / 2.  Adds to the element arrays and the
// patch adjoints.  One lane per (element, side): the two probes of an element
// sit in neighbouring lanes of one wave (work item 2 l + side) and trade their
// values with shuffles, so each lane evaluates two MLS fits, not four.
template <typename T>
__device__ void external_vjp(const AdjScratch<T>& S, const Patch<T>& P, int nv, double nu, int sx,
                             int sy, int& st)
{
    for (int w = threadIdx.x; w < 2 * nv; w += blockDim.x) {
        const int l = w >> 1, side = w & 1;
        const int m = l + 1 == nv ? 0 : l + 1;
        // probe support exactly as the forward kernel chose it (frame n-1)
        const T txT = (S.hxp[m] - S.hxp[l]) + (S.lxp[m] - S.lxp[l]);
        const T tyT = (S.hyp[m] - S.hyp[l]) + (S.lyp[m] - S.lyp[l]);
        const T lenT = sqrt(txT * txT + tyT * tyT);
        const T nxT = tyT / lenT, nyT = -txT / lenT;
        const T xcT = T(0.5) * (S.hxp[l] + S.hxp[m]), ycT = T(0.5) * (S.hyp[l] + S.hyp[m]);
        const T sgT = side ? T(-1.2) : T(1.2);
        const T pxT = xcT + sgT * nxT, pyT = ycT + sgT * nyT;
        const int cx = (int)floor(pxT + T(0.5)) + sx;
        const int cy = (int)floor(pyT + T(0.5)) + sy;
        // geometry in FP64 (patch frame)
        const double tx = S.Xp[m] - S.Xp[l], ty = S.Yp[m] - S.Yp[l];
        const double len = sqrt(tx * tx + ty * ty);
        const double npx = ty, npy = -tx;  // len * n+
        const double nx = npx / len, ny = npy / len;
        const double xc = 0.5 * (S.Xp[l] + S.Xp[m]), yc = 0.5 * (S.Yp[l] + S.Yp[m]);
        const double sg = side ? -1.2 : 1.2;
        const double px = xc + sg * nx, py = yc + sg * ny;
        // forward value of this lane's probe
        double r = 0, g00 = 0, g01 = 0, g10 = 0, g11 = 0;
        mls_dual<true>(px, py, cx, cy,
                       [&](int k, const Dual<2>& phi, const Dual<2>& gx, const Dual<2>& gy) {
                           const int idx = adj_patch_index(P, cx, cy, k);
                           if (idx < 0) { st |= ST_PATCH; return; }
                           const double u = S.pu[idx], v = S.pv[idx];
                           r += phi.v * (double)S.pd[idx];
                           g00 += gx.v * u;
                           g01 += gy.v * u;
                           g10 += gx.v * v;
                           g11 += gy.v * v;
                       });
        // both probes of the element: side 0 (outer) and side 1 (inner)
        const double own[5] = {r / 3.0, g00, g01, g10, g11};
        double pr[2][5];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            const double other = __shfl_xor(own[q], 1);
            pr[0][q] = side ? other : own[q];
            pr[1][q] = side ? own[q] : other;
        }
        const double dpr = pr[0][0] - pr[1][0];
        const double d00 = 2.0 * (pr[0][1] - pr[1][1]);
        const double d11 = 2.0 * (pr[0][4] - pr[1][4]);
        const double d01 = (pr[0][2] + pr[0][3]) - (pr[1][2] + pr[1][3]);
        const double hx = 0.5 * (S.lFx[l] + S.lFx[m]), hy = 0.5 * (S.lFy[l] + S.lFy[m]);
        // f = -dpr np + nu D np  (np = len n+, D symmetric)
        const double lnpx = -dpr * hx + nu * (d00 * hx + d01 * hy);
        const double lnpy = -dpr * hy + nu * (d01 * hx + d11 * hy);
        const double ldpr = -(npx * hx + npy * hy);
        const double ld00 = nu * hx * npx, ld11 = nu * hy * npy;
        const double ld01 = nu * (hx * npy + hy * npx);
        // reverse of this lane's probe
        const double sgn = side ? -1.0 : 1.0;
        const double lP = sgn * ldpr / 3.0;  // lambda of sum phi rho (p = rho / 3)
        const double l00 = 2.0 * sgn * ld00, l11 = 2.0 * sgn * ld11, l01 = sgn * ld01;
        double gpx = 0.0, gpy = 0.0;
        mls_dual<true>(px, py, cx, cy,
                       [&](int k, const Dual<2>& phi, const Dual<2>& gx, const Dual<2>& gy) {
                           const int idx = adj_patch_index(P, cx, cy, k);
                           if (idx < 0) return;
                           const double d = S.pd[idx], u = S.pu[idx], v = S.pv[idx];
                           // G00 = sum gx u, G01 = sum gy u, G10 = sum gx v, G11 = sum gy v
                           const double cgx = l00 * u + l01 * v;
                           const double cgy = l01 * u + l11 * v;
                           gpx += lP * d * phi.d[0] + cgx * gx.d[0] + cgy * gy.d[0];
                           gpy += lP * d * phi.d[1] + cgx * gx.d[1] + cgy * gy.d[1];
                           atomicAdd(&S.Ld[idx], (T)(lP * phi.v));
                           atomicAdd(&S.Lu[idx], (T)(l00 * gx.v + l01 * gy.v));
                           atomicAdd(&S.Lv[idx], (T)(l01 * gx.v + l11 * gy.v));
                       });
        // sums over the two probes (side 0 first)
        const double ox = __shfl_xor(gpx, 1), oy = __shfl_xor(gpy, 1);
        if (side) continue;
        const double lxc = gpx + ox, lyc = gpy + oy;
        const double lnx = 1.2 * gpx + -1.2 * ox, lny = 1.2 * gpy + -1.2 * oy;
        double ltx = -lnpy, lty = lnpx;  // np = (t_y, -t_x)
        // n = R t / len: (dn/dt)^T v = ((-v_y, v_x) - t^ (n . v)) / len
        const double ndot = nx * lnx + ny * lny;
        ltx += (-lny - tx / len * ndot) / len;
        lty += (lnx - ty / len * ndot) / len;
        S.E1x[l] += 0.5 * lxc - ltx;
        S.E1y[l] += 0.5 * lyc - lty;
        S.E2x[l] += 0.5 * lxc + ltx;
        S.E2y[l] += 0.5 * lyc + lty;
    }
}

// One block per capsule: reverse of one IB launch of the forward run.
//   doB    the node update closing step n-1 (Dynamic: Eqs. 21-24 with the
//          internal and hydrodynamic forces; Kinematic: Eq. 25)
//   prime  the start-up u_v^0 = d^0 = U(x^0) (n = 0)
//   doA    the forcing of step n (Dynamic direct forcing with c_v = arc
//          length; Kinematic internal forces with c_v = 1) and its spreading
// Carried adjoints lamx, lamd enter as those of x^n, d^n and leave as those
// of x^{n-1}, d^{n-1}.  The adjoint of the moments M^n goes into lambda P^n
// (transpose of the pull) and lambda F^{n-1} (its half-force term).
// One instance per coupling (DYN = a.dynamic), as the forward IB kernel, and
// per bending (BEND = a.bend: some capsule has k_b != 0; without it the
// bending terms are compiled out, which keeps the Kinematic instance 1 us
// shorter per reverse step).
template <typename T, bool DYN, bool BEND>
__global__ __launch_bounds__(kAdjThreads) void k_ib_adj(IBAdjArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kIBThreads / 64][8];
    const int tid = threadIdx.x, nt = blockDim.x, c = blockIdx.x;
    const CapsuleDev cap = a.caps[c];
    const int nv = cap.nv, off = cap.node_offset;
    const size_t NS = a.stride;
    GridArgs g;
    g.nx = cap.nx;
    g.ny = cap.ny;
    g.nxp = cap.nxp;
    g.nseg = cap.nseg;
    g.periodic_y = cap.periodic_y;
    g.periodic_x = cap.periodic_x;
    g.omega = 0.0;
    g.gx = cap.gx;
    g.u_bot = g.u_top = 0.0;
    g.u_in = 0.0;
    g.rho_out = 1.0;
    g.uref_c = cap.uref_c;
    const size_t plane = (size_t)g.ny * g.nxp;
    T* lam_p = a.lam_p + cap.pop_off;
    T* lfm = a.lfm + cap.fib_off;
    int* lfm_flags = a.lfm_flags + cap.flag_off;
    const T* lft = a.lft + cap.fib_off;

    AdjScratch<T> S;
    {
        T* p = reinterpret_cast<T*>(smem);
        const int pc = a.patch_cap, M = a.max_nv;
        S.pd = p; S.pu = p + pc; S.pv = p + 2 * pc;
        S.Ld = p + 3 * pc; S.Lu = p + 4 * pc; S.Lv = p + 5 * pc;
        T* q = p + 6 * pc;
        S.hxn = q; S.hyn = q + M; S.hxp = q + 2 * M; S.hyp = q + 3 * M;
        S.lxp = q + 4 * M; S.lyp = q + 5 * M;
        size_t b = sizeof(T) * ((size_t)kAdjRealCellArrays * pc + (size_t)kAdjRealNodeArrays * M);
        b = (b + 15) & ~(size_t)15;
        double* d = reinterpret_cast<double*>(smem + b);
        double** arr[kAdjDoubleArrays] = {&S.Xn, &S.Yn, &S.Xp, &S.Yp, &S.uvx, &S.uvy, &S.lx, &S.ly,
                                          &S.ldx, &S.ldy, &S.lux, &S.luy, &S.lFx, &S.lFy, &S.lc,
                                          &S.E1x, &S.E1y, &S.E2x, &S.E2y, &S.Fvx, &S.Fvy};
        for (int k = 0; k < kAdjDoubleArrays; k++) *arr[k] = d + (size_t)k * M;
    }

    // reference points of the two time levels; x^{n-1} is moved to frame n
    const double rnx = a.ref_n[2 * c], rny = a.ref_n[2 * c + 1];
    const double rpx = a.doB ? a.ref_p[2 * c] : rnx, rpy = a.doB ? a.ref_p[2 * c + 1] : rny;
    const int sx = (int)(rpx - rnx), sy = (int)(rpy - rny);
    const T* Nn = a.nodes_n;
    const T* Np = a.nodes_p;
    float mn[2] = {3e38f, 3e38f}, mxv[2] = {-3e38f, -3e38f};
    for (int v = tid; v < nv; v += nt) {
        const T hx = Nn[NF_HX * NS + off + v], hy = Nn[NF_HY * NS + off + v];
        S.hxn[v] = hx;
        S.hyn[v] = hy;
        S.Xn[v] = (double)hx + (double)Nn[NF_LX * NS + off + v];
        S.Yn[v] = (double)hy + (double)Nn[NF_LY * NS + off + v];
        S.uvx[v] = (double)Nn[NF_UX * NS + off + v];
        S.uvy[v] = (double)Nn[NF_UY * NS + off + v];
        mn[0] = fminf(mn[0], (float)S.Xn[v]);
        mn[1] = fminf(mn[1], (float)S.Yn[v]);
        mxv[0] = fmaxf(mxv[0], (float)S.Xn[v]);
        mxv[1] = fmaxf(mxv[1], (float)S.Yn[v]);
        if (a.doB) {
            const T px = Np[NF_HX * NS + off + v], py = Np[NF_HY * NS + off + v];
            const T qx = Np[NF_LX * NS + off + v], qy = Np[NF_LY * NS + off + v];
            S.hxp[v] = px;
            S.hyp[v] = py;
            S.lxp[v] = qx;
            S.lyp[v] = qy;
            S.Xp[v] = (double)px + (double)qx + (double)sx;
            S.Yp[v] = (double)py + (double)qy + (double)sy;
            mn[0] = fminf(mn[0], (float)S.Xp[v]);
            mn[1] = fminf(mn[1], (float)S.Yp[v]);
            mxv[0] = fmaxf(mxv[0], (float)S.Xp[v]);
            mxv[1] = fmaxf(mxv[1], (float)S.Yp[v]);
        }
        S.lx[v] = a.lamx[off + v];
        S.ly[v] = a.lamx[NS + off + v];
        S.ldx[v] = a.lamd[off + v];
        S.ldy[v] = a.lamd[NS + off + v];
        S.lux[v] = S.luy[v] = 0.0;
        S.lFx[v] = S.lFy[v] = S.lc[v] = 0.0;
        S.E1x[v] = S.E1y[v] = S.E2x[v] = S.E2y[v] = 0.0;
    }
    block_minmax(mn, mxv, red);
    if (!(mn[0] > -1e6f && mxv[0] < 1e6f && mn[1] > -1e6f && mxv[1] < 1e6f)) {
        if (tid == 0) atomicOr(a.status, ST_NONFINITE);
        return;
    }
    Patch<T> P;
    P.drho = S.pd;
    P.ux = S.pu;
    P.uy = S.pv;
    P.ox = (int)floorf(mn[0]) - 3;
    P.oy = (int)floorf(mn[1]) - 3;
    P.W = (int)floorf(mxv[0]) - (int)floorf(mn[0]) + 7;
    P.H = (int)floorf(mxv[1]) - (int)floorf(mn[1]) + 7;
    if ((long long)P.W * P.H > a.patch_cap) {
        if (tid == 0) atomicOr(a.status, ST_PATCH);
        return;
    }
    const long long refx = (long long)rnx, refy = (long long)rny;
    // the reference point on the periodic axes (x always periodic here)
    const int wrx = wrap_ref(refx, g.nx), wry = g.periodic_y ? wrap_ref(refy, g.ny) : 0;
    {
        IBArgs<T> ia;
        ia.pops = a.pops + cap.pop_off;
        ia.fib_prev = a.fib_prev + cap.fib_off;
        const T gxf = (T)cap.gx;
        const int ncell = P.W * P.H;
        // four cells per thread with all their loads in flight together
        for (int i = tid; i < ncell; i += 4 * nt) stage_cells<T, 4>(ia, g, P, refx, refy, gxf, i, nt);
        for (int i = tid; i < ncell; i += nt) S.Ld[i] = S.Lu[i] = S.Lv[i] = T(0);
    }
    __syncthreads();
    int st = 0;
    const double nu = cap.nu;

    // ---- reverse of the forcing of step n (at x^n)
    if (a.doA) {
        if (DYN) {
            for (int v = tid; v < nv; v += nt) {
                const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
                const int cx = (int)floor(S.hxn[v] + T(0.5)), cy = (int)floor(S.hyn[v] + T(0.5));
                double ph[9], phx[9], phy[9];
                int id9[9];
                double Ux = 0, Uy = 0;
                mls_dual<false>(S.Xn[v], S.Yn[v], cx, cy,
                                [&](int k, const Dual<2>& phi, const Dual<2>&, const Dual<2>&) {
                                    ph[k] = phi.v;
                                    phx[k] = phi.d[0];
                                    phy[k] = phi.d[1];
                                    id9[k] = adj_patch_index(P, cx, cy, k);
                                    if (id9[k] >= 0) {
                                        Ux += phi.v * (double)S.pu[id9[k]];
                                        Uy += phi.v * (double)S.pv[id9[k]];
                                    }
                                });
                const double Fx = S.uvx[v] - Ux, Fy = S.uvy[v] - Uy;
                const double ax = S.Xn[v] - S.Xn[vl], ay = S.Yn[v] - S.Yn[vl];
                const double bx = S.Xn[vr] - S.Xn[v], by = S.Yn[vr] - S.Yn[v];
                const double cv = 0.5 * (sqrt(ax * ax + ay * ay) + sqrt(bx * bx + by * by));
                double lfk[9][2];
                double sLx = 0, sLy = 0, lcv = 0;
                for (int k = 0; k < 9; k++) {
                    lfk[k][0] = lfk[k][1] = 0.0;
                    int gy;
                    if (g.periodic_y) {
                        gy = wrap_add(wry, cy + k / 3 - 1, g.ny);
                    } else {
                        const long long yv = refy + cy + k / 3 - 1;
                        if (yv < 1 || yv > g.ny - 2) continue;
                        gy = (int)yv;
                    }
                    const int gxx = wrap_add(wrx, cx + k % 3 - 1, g.nx);
                    const size_t cell = (size_t)gy * g.nxp + (size_t)gxx;
                    lfk[k][0] = (double)lft[2 * cell];
                    lfk[k][1] = (double)lft[2 * cell + 1];
                    sLx += ph[k] * lfk[k][0];
                    sLy += ph[k] * lfk[k][1];
                    lcv += ph[k] * (Fx * lfk[k][0] + Fy * lfk[k][1]);
                }
                const double lFvx = cv * sLx, lFvy = cv * sLy;
                double gpx = 0, gpy = 0;
                for (int k = 0; k < 9; k++) {
                    const int idx = id9[k];
                    const double u = idx >= 0 ? (double)S.pu[idx] : 0.0;
                    const double w = idx >= 0 ? (double)S.pv[idx] : 0.0;
                    const double lph = cv * (Fx * lfk[k][0] + Fy * lfk[k][1]) - (u * lFvx + w * lFvy);
                    gpx += lph * phx[k];
                    gpy += lph * phy[k];
                    if (idx >= 0) {
                        atomicAdd(&S.Lu[idx], (T)(-ph[k] * lFvx));
                        atomicAdd(&S.Lv[idx], (T)(-ph[k] * lFvy));
                    } else {
                        st |= ST_PATCH;
                    }
                }
                S.lx[v] += gpx;
                S.ly[v] += gpy;
                S.lux[v] = lFvx;
                S.luy[v] = lFvy;
                S.lc[v] = lcv;
            }
            __syncthreads();
            for (int v = tid; v < nv; v += nt) {
                const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
                const double ax = S.Xn[v] - S.Xn[vl], ay = S.Yn[v] - S.Yn[vl];
                const double bx = S.Xn[vr] - S.Xn[v], by = S.Yn[vr] - S.Yn[v];
                const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
                const double ca = 0.5 * (S.lc[v] + S.lc[vl]), cb = 0.5 * (S.lc[v] + S.lc[vr]);
                S.lx[v] += ca * ax / la - cb * bx / lb;
                S.ly[v] += ca * ay / la - cb * by / lb;
            }
            __syncthreads();
        } else {
            const T* N0 = a.consts;
            internal_fwd<BEND>(S, S.Xn, S.Yn, nv, N0 + NF_L0 * NS + off, N0 + NF_L0L * NS + off,
                         N0 + NF_KS * NS + off, cap.kb, N0 + NF_TH0 * NS + off, cap.ka, cap.A0,
                         red);
            for (int v = tid; v < nv; v += nt) {
                const int cx = (int)floor(S.hxn[v] + T(0.5)), cy = (int)floor(S.hyn[v] + T(0.5));
                double lFvx = 0, lFvy = 0, gpx = 0, gpy = 0;
                const double Fx = S.Fvx[v], Fy = S.Fvy[v];
                mls_dual<false>(S.Xn[v], S.Yn[v], cx, cy,
                                [&](int k, const Dual<2>& phi, const Dual<2>&, const Dual<2>&) {
                                    int gy;
                                    if (g.periodic_y) {
                                        gy = wrap_add(wry, cy + k / 3 - 1, g.ny);
                                    } else {
                                        const long long yv = refy + cy + k / 3 - 1;
                                        if (yv < 1 || yv > g.ny - 2) return;
                                        gy = (int)yv;
                                    }
                                    const int gxx = wrap_add(wrx, cx + k % 3 - 1, g.nx);
                                    const size_t cell = (size_t)gy * g.nxp + (size_t)gxx;
                                    const double lx_ = (double)lft[2 * cell];
                                    const double ly_ = (double)lft[2 * cell + 1];
                                    lFvx += phi.v * lx_;
                                    lFvy += phi.v * ly_;
                                    const double lph = Fx * lx_ + Fy * ly_;
                                    gpx += lph * phi.d[0];
                                    gpy += lph * phi.d[1];
                                });
                S.lx[v] += gpx;
                S.ly[v] += gpy;
                S.lFx[v] = lFvx;
                S.lFy[v] = lFvy;
            }
            __syncthreads();
            const T* N1 = a.consts;
            const double lA = internal_vjp<BEND>(S, S.Xn, S.Yn, nv, N1 + NF_L0 * NS + off,
                                           N1 + NF_L0L * NS + off, N1 + NF_KS * NS + off, cap.kb,
                                           N1 + NF_TH0 * NS + off, cap.ka, cap.A0, a.ksbar + off,
                                           red);
            __syncthreads();
            for (int v = tid; v < nv; v += nt) {
                const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
                S.lx[v] += S.E1x[v] + S.E2x[vl] + lA * 0.5 * (S.Yn[vr] - S.Yn[vl]);
                S.ly[v] += S.E1y[v] + S.E2y[vl] + lA * 0.5 * (S.Xn[vl] - S.Xn[vr]);
                S.lFx[v] = S.lFy[v] = 0.0;
            }
            __syncthreads();
            for (int v = tid; v < nv; v += nt) S.E1x[v] = S.E1y[v] = S.E2x[v] = S.E2y[v] = 0.0;
            __syncthreads();
        }
    }

    // ---- reverse of the start-up: u_v^0 = d^0 = U(x^0)
    if (a.prime) {
        for (int v = tid; v < nv; v += nt) {
            const int cx = (int)floor(S.hxn[v] + T(0.5)), cy = (int)floor(S.hyn[v] + T(0.5));
            const double lUx = S.lux[v] + S.ldx[v], lUy = S.luy[v] + S.ldy[v];
            double gpx, gpy;
            interp_vjp(S, P, S.Xn[v], S.Yn[v], cx, cy, lUx, lUy, gpx, gpy, st);
            S.lx[v] += gpx;
            S.ly[v] += gpy;
            S.ldx[v] = S.ldy[v] = 0.0;
        }
        __syncthreads();
    }

    // ---- reverse of the node update closing step n-1 (at x^{n-1})
    if (a.doB) {
        const double m = cap.mv;
        for (int v = tid; v < nv; v += nt) {
            double lvx, lvy;  // adjoint of the interpolated velocity (xdot_0 / xdot)
            if (DYN) {
                const double tx = S.ldx[v] + 1.5 * S.lux[v] + S.lx[v];
                const double ty = S.ldy[v] + 1.5 * S.luy[v] + S.ly[v];
                S.lFx[v] = tx / (2.0 * m);
                S.lFy[v] = ty / (2.0 * m);
                S.ldx[v] = -0.5 * S.lux[v];
                S.ldy[v] = -0.5 * S.luy[v];
                lvx = tx;
                lvy = ty;
            } else {
                const double tx = S.ldx[v] + S.lx[v], ty = S.ldy[v] + S.ly[v];
                S.ldx[v] = tx / 3.0;
                S.ldy[v] = ty / 3.0;
                lvx = 2.0 * tx / 3.0;
                lvy = 2.0 * ty / 3.0;
            }
            const int cx = (int)floor(S.hxp[v] + T(0.5)) + sx;
            const int cy = (int)floor(S.hyp[v] + T(0.5)) + sy;
            double gpx, gpy;
            interp_vjp(S, P, S.Xp[v], S.Yp[v], cx, cy, lvx, lvy, gpx, gpy, st);
            S.lx[v] += gpx;
            S.ly[v] += gpy;
        }
        __syncthreads();
        if (DYN) {
            const T* N0 = a.consts;
            const double lA = internal_vjp<BEND>(S, S.Xp, S.Yp, nv, N0 + NF_L0 * NS + off,
                                           N0 + NF_L0L * NS + off, N0 + NF_KS * NS + off, cap.kb,
                                           N0 + NF_TH0 * NS + off, cap.ka, cap.A0, a.ksbar + off,
                                           red);
            external_vjp(S, P, nv, nu, sx, sy, st);
            __syncthreads();
            for (int v = tid; v < nv; v += nt) {
                const int vl = v == 0 ? nv - 1 : v - 1, vr = v + 1 == nv ? 0 : v + 1;
                S.lx[v] += S.E1x[v] + S.E2x[vl] + lA * 0.5 * (S.Yp[vr] - S.Yp[vl]);
                S.ly[v] += S.E1y[v] + S.E2y[vl] + lA * 0.5 * (S.Xp[vl] - S.Xp[vr]);
            }
        }
        __syncthreads();
    }

    for (int v = tid; v < nv; v += nt) {
        a.lamx[off + v] = S.lx[v];
        a.lamx[NS + off + v] = S.ly[v];
        a.lamd[off + v] = S.ldx[v];
        a.lamd[NS + off + v] = S.ldy[v];
    }

    // ---- moments adjoint -> lambda P^n (transpose of the pull), lambda F^{n-1}
    {
        const int ncell = P.W * P.H;
        const int pbx = wrap_ref(refx + P.ox, g.nx);
        const int pby = g.periodic_y ? wrap_ref(refy + P.oy, g.ny) : 0;
        for (int i = tid; i < ncell; i += nt) {
            const T Ld = S.Ld[i], Lu = S.Lu[i], Lv = S.Lv[i];
            if (Ld == T(0) && Lu == T(0) && Lv == T(0)) continue;
            if (isnan(S.pd[i])) continue;
            const int lxi = i % P.W, lyi = i / P.W;
            const long long wy = g.periodic_y ? (long long)wrap_add(pby, lyi, g.ny)
                                              : refy + P.oy + lyi;
            const int wx = wrap_add(pbx, lxi, g.nx);
            const T rho = T(1) + S.pd[i];
            const T ux = S.pu[i], uy = S.pv[i];
            const T irho = T(1) / rho;
            const int x = (int)wx, y = (int)wy;
            const int xm = x == 0 ? g.nx - 1 : x - 1;
            const int xp = x == g.nx - 1 ? 0 : x + 1;
            for (int q = 0; q < 9; q++) {
                const T ls = Ld + (((T)kEx[q] - ux) * Lu + ((T)kEy[q] - uy) * Lv) * irho;
                const int xs = kEx[q] > 0 ? xm : (kEx[q] < 0 ? xp : x);
                int ys = y - kEy[q];
                if (g.periodic_y) ys = ys < 0 ? g.ny - 1 : (ys >= g.ny ? 0 : ys);
                atomicAdd(&lam_p[q * plane + (size_t)ys * g.nxp + xs], ls);
            }
            const size_t cell = (size_t)y * g.nxp + x;
            atomicAdd(&lfm[2 * cell], T(0.5) * Lu * irho);
            atomicAdd(&lfm[2 * cell + 1], T(0.5) * Lv * irho);
            lfm_flags[y * g.nseg + x / kSegW] = 1;
        }
    }
    if (st) atomicOr(a.status, st);
}

// ------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_grid_adj(const GridAdjArgs<T>& a, const GridArgs& g, hipStream_t s)
{
    const int blocks = grid_blocks(g.ny, g.nseg);
    hipLaunchKernelGGL(k_grid_adj<T>, dim3(blocks), dim3(kSegW * 4), 0, s, a, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_adj(const GridAdjArgs<T>& a, const GridArgs& g, int profile, double nu,
                           hipStream_t s)
{
    const int blocks = grid_blocks(g.ny, g.nseg);
    hipLaunchKernelGGL(k_init_adj<T>, dim3(blocks), dim3(kSegW * 4), 0, s, a, g, profile, nu);
    return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* v, int n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kIBThreads), 0, s, v, n, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_seed(const T* nodes, const double* ref, const CapsuleDev* caps, int cap_id,
                           int stride, int objective, double* lamx, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_seed<T>, dim3(1), dim3(kIBThreads), 0, s, nodes, ref, caps, cap_id,
                       stride, objective, lamx, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ib_adj(const IBAdjArgs<T>& a, int ncap, size_t lds_bytes, hipStream_t s)
{
    if (ncap <= 0) return hipSuccess;
    const dim3 grid(ncap), block(kAdjThreads);
    if (a.dynamic) {
        if (a.bend)
            hipLaunchKernelGGL((k_ib_adj<T, true, true>), grid, block, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_ib_adj<T, true, false>), grid, block, lds_bytes, s, a);
    } else {
        if (a.bend)
            hipLaunchKernelGGL((k_ib_adj<T, false, true>), grid, block, lds_bytes, s, a);
        else
            hipLaunchKernelGGL((k_ib_adj<T, false, false>), grid, block, lds_bytes, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t ib_adj_set_lds_limit(size_t bytes)
{
    const void* fns[4] = {reinterpret_cast<const void*>(&k_ib_adj<T, true, false>),
                          reinterpret_cast<const void*>(&k_ib_adj<T, false, false>),
                          reinterpret_cast<const void*>(&k_ib_adj<T, true, true>),
                          reinterpret_cast<const void*>(&k_ib_adj<T, false, true>)};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define LBIB_ADJ_INST(T)                                                                          \
    template hipError_t launch_grid_adj<T>(const GridAdjArgs<T>&, const GridArgs&, hipStream_t);  \
    template hipError_t launch_init_adj<T>(const GridAdjArgs<T>&, const GridArgs&, int, double,   \
                                           hipStream_t);                                          \
    template hipError_t launch_adj_seed<T>(const T*, const double*, const CapsuleDev*, int, int,  \
                                           int, double*, double*, hipStream_t);                   \
    template hipError_t launch_ib_adj<T>(const IBAdjArgs<T>&, int, size_t, hipStream_t);          \
    template hipError_t ib_adj_set_lds_limit<T>(size_t);                                          \
    template size_t ib_adj_lds_bytes<T>(int, int);

LBIB_ADJ_INST(float)
LBIB_ADJ_INST(double)

}  // namespace lbib
