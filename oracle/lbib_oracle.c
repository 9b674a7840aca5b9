/*
 * FP64 CPU oracle for the lattice Boltzmann - Kinematic / Dynamic immersed
 * boundary method for deformable capsules (Coclite et al., arXiv:1903.03356).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does.  It
 * shares no code, header, table or constant with the HIP sources.
 *
 * Everything is double precision, in the paper's order and notation:
 *   Sec. 2.1   D2Q9 BGK lattice Boltzmann, Eqs. 1-3, Zou-He walls
 *   Sec. 2.2   Guo forcing, Eqs. 4-7; MLS transfer, Eqs. 8-9
 *   Sec. 2.2.1 membrane forces, Eqs. 10-14
 *   Sec. 2.2.2 hydrodynamic stresses, Eqs. 15-16
 *   Sec. 2.3.2 Dynamic IB: Newton/Verlet node update, Eqs. 21-24, steps 1-8
 *   Sec. 2.4   Kinematic IB, steps i-viii, Eq. 25
 *   Sec. 3     diagnostics: Taylor deformation, perimeter change, swelling ratio
 *
 * Readings where the paper is silent, garbled or inconsistent are marked
 * "reading:" at the point of use.
 *
 * Layout (private to this file): populations f[(x * ny + y) * 9 + i], fields
 * [x * ny + y].  The public get/set calls convert to [component][y][x].
 *
 * Parity status of each function is recorded next to it: every function is
 * pinned by a CPU test except where the comment says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Lattice (Eq. 3).  Rest velocity, then the four axis directions at angles
 * (i-1) pi/2 (E, N, W, S), then the diagonals sqrt(2)(cos, sin)((2i-9) pi/4)
 * (NE, NW, SW, SE).  Weights 4/9, 1/9, 1/36.  c_s^2 = 1/3.
 * ------------------------------------------------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* MLS constants (Sec. 2.2, Eq. 9): support side r_w = 2.6 dx, alpha = 0.3 */
static const double MLS_RW = 2.6;
static const double MLS_ALPHA = 0.3;
/* hydrodynamic probe length along the element normal (Sec. 2.2.2) */
static const double PROBE_LEN = 1.2;

enum { ORC_KINEMATIC = 0, ORC_DYNAMIC = 1 };
enum { ORC_E_WALL = 1, ORC_E_NONFINITE = 2 };

typedef struct {
    int nv;
    double *x;      /* x^n, [2 nv] */
    double *xm1;    /* x^{n-1} */
    double *uv;     /* u_v^n (Eq. 24), Dynamic only */
    double *l0;     /* stress-free element lengths, element l joins node l to l+1 */
    double *theta0; /* stress-free turning angle at each node */
    double *ks;     /* per-element stretching constant */
    double kb, ka, mass, mv, A0, P0;
    double *ftot;   /* last total nodal force (Dynamic) or internal force (Kinematic) */
    double *fext;   /* last hydrodynamic nodal force (Dynamic) */
    double *fc;     /* contact force of the current positions (Eq. 27) */
    int primed;
    /* rigid particle (Sec. 2.3.1): nodes x_v = X + R(theta) r0_v */
    int rigid;
    double *r0;               /* body-frame offsets from the area centroid, [2 nv] */
    double X[2], theta;       /* centroid and rotation angle */
    double u[2], um1[2];      /* velocity at n and n-1 (Eq. 19) */
    double w, wm1;            /* angular velocity at n and n-1 (Eq. 20) */
    double I;                 /* moment of inertia about the centroid */
    double Ftot[2], Mtot;     /* last hydrodynamic force and torque (Eqs. 17-18) */
} orc_capsule;

typedef struct {
    int nx, ny, periodic_y;
    int periodic_x;            /* 0: velocity inlet at x = 0, pressure outlet at x = nx-1 */
    double u_in, rho_out;      /* inlet peak speed (parabolic profile), outlet density */
    double tau, nu;
    double u_bot, u_top, gx, gy;
    double *f, *ftmp;          /* [nx][ny][9] */
    double *F;                 /* total force of the last collision, F^{n-1}: [nx][ny][2] */
    double *fib;               /* IB force being assembled: [nx][ny][2] */
    double *rho, *ux, *uy;     /* moments of f with half of F: [nx][ny] */
    int ncap, capcap;
    orc_capsule *caps;
    long steps;
    int mode;                  /* -1 until the first step */
    int status;
    double contact_cutoff;     /* Eq. 27 repulsion acts below this distance; 0 = off */
} orc_sim;

static inline size_t cid(const orc_sim *s, int x, int y) { return (size_t)x * s->ny + y; }
static inline int wrap(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* ---------------------------------------------------------------------------
 * Eq. 2: second-order equilibrium, c_s^2 = 1/3.
 * Pinned: moment identities (sum = rho, first moment = rho u, second moment
 * rho (c_s^2 I + u u)).
 * ------------------------------------------------------------------------- */
void orc_equilibrium(double rho, double ux, double uy, double feq[9])
{
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = WGT[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    }
}

/* ---------------------------------------------------------------------------
 * Eq. 5: forcing term (Guo form)
 *   F_i = (1 - 1/(2 tau)) w_i [ (e_i - u)/c_s^2 + (e_i . u) e_i / c_s^4 ] . f
 * Pinned: zeroth moment 0, first moment (1 - 1/(2 tau)) f.
 * ------------------------------------------------------------------------- */
void orc_forcing(double tau, double ux, double uy, double fx, double fy, double out[9])
{
    double pre = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        double vx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
        double vy = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
        out[i] = pre * WGT[i] * (vx * fx + vy * fy);
    }
}

/* ---------------------------------------------------------------------------
 * Eq. 9: MLS shape functions at a point (xm, ym).
 * Support: the 3x3 lattice nodes centred on the node nearest the point
 * (reading: nearest = floor(x + 1/2), ties go up).  Cell k = 3 (dy+1) + (dx+1).
 * Weight W_k = exp(-(r_k/alpha)^2), r_k = |x - x_k| / r_w.
 * Linear basis p = [1, x - xm, y - ym] (reading: centred on the point, which
 * spans the same space as [1, x, y]).  A = sum_k W_k p_k p_k^T; the fit
 * coefficients are a = A^{-1} sum_k W_k p_k u_k, so
 *   phi_k   = (A^{-1} W_k p_k)[0]   (value at the point, Eq. 8)
 *   dphix_k = (A^{-1} W_k p_k)[1],  dphiy_k = (A^{-1} W_k p_k)[2]
 * (reading: velocity derivatives are the slope coefficients of the local fit).
 * The 3x3 system is solved by Gaussian elimination with partial pivoting.
 * Pinned: partition of unity, exact reproduction of linear fields and their
 * gradients, closed form W/sum(W) for a point on a node.
 * ------------------------------------------------------------------------- */
void orc_mls(double xm, double ym, int cx[9], int cy[9], double phi[9], double dphix[9],
             double dphiy[9])
{
    int ix = (int)floor(xm + 0.5), iy = (int)floor(ym + 0.5);
    double p[9][3], w[9];
    double A[3][3] = {{0}};
    for (int k = 0; k < 9; k++) {
        int dx = k % 3 - 1, dy = k / 3 - 1;
        cx[k] = ix + dx;
        cy[k] = iy + dy;
        double rx = cx[k] - xm, ry = cy[k] - ym;
        double r = sqrt(rx * rx + ry * ry) / MLS_RW;
        w[k] = exp(-(r / MLS_ALPHA) * (r / MLS_ALPHA));
        p[k][0] = 1.0;
        p[k][1] = rx;
        p[k][2] = ry;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) A[a][b] += w[k] * p[k][a] * p[k][b];
    }
    /* right-hand sides B[:, k] = W_k p_k; solve A X = B */
    double M[3][3 + 9];
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) M[a][b] = A[a][b];
        for (int k = 0; k < 9; k++) M[a][3 + k] = w[k] * p[k][a];
    }
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 12; j++) {
                double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
        for (int r = 0; r < 3; r++) {
            if (r == c) continue;
            double m = M[r][c] / M[c][c];
            for (int j = 0; j < 12; j++) M[r][j] -= m * M[c][j];
        }
    }
    for (int k = 0; k < 9; k++) {
        phi[k] = M[0][3 + k] / M[0][0];
        dphix[k] = M[1][3 + k] / M[1][1];
        dphiy[k] = M[2][3 + k] / M[2][2];
    }
}

/* ---------------------------------------------------------------------------
 * Geometry helpers on a closed polygon of nv nodes, counter-clockwise.
 * Element l joins node l to node l+1 (mod nv).  Reading: outward normal of an
 * element with tangent t = x_{l+1} - x_l is n+ = (t_y, -t_x)/|t|, n- = -n+.
 * ------------------------------------------------------------------------- */
static double polygon_area(int nv, const double *x)
{
    /* Green's theorem, A = 1/2 closed integral of (x dy - y dx) (Sec. 2.2.1;
     * reading: the printed formula lacks the 1/2) */
    double a = 0.0;
    for (int l = 0; l < nv; l++) {
        int m = (l + 1) % nv;
        a += x[2 * l] * x[2 * m + 1] - x[2 * m] * x[2 * l + 1];
    }
    return 0.5 * a;
}

static double turning_angle(int nv, const double *x, int v)
{
    /* reading: the angle at node v between its two edges is the signed
     * turning angle from a = x_v - x_{v-1} to b = x_{v+1} - x_v */
    int vl = (v + nv - 1) % nv, vr = (v + 1) % nv;
    double ax = x[2 * v] - x[2 * vl], ay = x[2 * v + 1] - x[2 * vl + 1];
    double bx = x[2 * vr] - x[2 * v], by = x[2 * vr + 1] - x[2 * v + 1];
    return atan2(ax * by - ay * bx, ax * bx + ay * by);
}

/* ---------------------------------------------------------------------------
 * Eqs. 10-14: internal (membrane) nodal forces.  Outputs are accumulated into
 * fs (stretch), fb (bending), fa (area), each [2 nv], zeroed here.
 *
 * Stretch, Eq. 11: F_v1 = -k_s (l - l0) r_12 / l, F_v2 = -k_s (l - l0) r_21 / l.
 *
 * Bending, Eq. 13.  Reading: the outer terms are used as printed,
 *   F_vleft  = k_b sin(theta - theta0) n_left  / l_left
 *   F_vright = k_b sin(theta - theta0) n_right / l_right
 * and the middle node takes minus their sum (the printed middle term is not
 * consistent with a force balance).  With theta the signed turning angle and
 * outward normals this is exactly minus the gradient of
 * k_b sum_v (1 - cos(theta_v - theta0_v)).
 *
 * Area, Eq. 14: F_l = -k_a (1 - A/A0) p_ref n-_l l_l, p_ref = rho_ref c_s^2,
 * half of F_l to each end node of element l.
 *
 * Pinned: zero net force and torque, zero at the stress-free state,
 * stretch and bending equal minus the gradient of their energies.
 * ------------------------------------------------------------------------- */
void orc_internal_forces(int nv, const double *x, const double *l0, const double *theta0,
                         const double *ks, double kb, double ka, double A0, double *fs,
                         double *fb, double *fa)
{
    memset(fs, 0, sizeof(double) * 2 * nv);
    memset(fb, 0, sizeof(double) * 2 * nv);
    memset(fa, 0, sizeof(double) * 2 * nv);
    const double p_ref = 1.0 * CS2;
    double A = polygon_area(nv, x);
    for (int l = 0; l < nv; l++) {
        int v1 = l, v2 = (l + 1) % nv;
        double r12x = x[2 * v1] - x[2 * v2], r12y = x[2 * v1 + 1] - x[2 * v2 + 1];
        double len = sqrt(r12x * r12x + r12y * r12y);
        double c = -ks[l] * (len - l0[l]) / len;
        fs[2 * v1] += c * r12x;
        fs[2 * v1 + 1] += c * r12y;
        fs[2 * v2] += -c * r12x;
        fs[2 * v2 + 1] += -c * r12y;

        double tx = -r12x, ty = -r12y; /* x_{v2} - x_{v1} */
        double nmx = -ty / len, nmy = tx / len; /* inward normal n- */
        double fmag = -ka * (1.0 - A / A0) * p_ref * len;
        fa[2 * v1] += 0.5 * fmag * nmx;
        fa[2 * v1 + 1] += 0.5 * fmag * nmy;
        fa[2 * v2] += 0.5 * fmag * nmx;
        fa[2 * v2 + 1] += 0.5 * fmag * nmy;
    }
    if (kb != 0.0) {
        for (int v = 0; v < nv; v++) {
            int vl = (v + nv - 1) % nv, vr = (v + 1) % nv;
            double ax = x[2 * v] - x[2 * vl], ay = x[2 * v + 1] - x[2 * vl + 1];
            double bx = x[2 * vr] - x[2 * v], by = x[2 * vr + 1] - x[2 * v + 1];
            double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
            double nLx = ay / la, nLy = -ax / la; /* outward normal of the left edge */
            double nRx = by / lb, nRy = -bx / lb; /* outward normal of the right edge */
            double sn = sin(turning_angle(nv, x, v) - theta0[v]);
            double FLx = kb * sn * nLx / la, FLy = kb * sn * nLy / la;
            double FRx = kb * sn * nRx / lb, FRy = kb * sn * nRy / lb;
            fb[2 * vl] += FLx;
            fb[2 * vl + 1] += FLy;
            fb[2 * vr] += FRx;
            fb[2 * vr + 1] += FRy;
            fb[2 * v] -= FLx + FRx;
            fb[2 * v + 1] -= FLy + FRy;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Sec. 3.1-3.2 diagnostics of a closed polygon:
 *   out[0] area (Green), out[1] perimeter, out[2..3] area centroid,
 *   out[4] Taylor deformation D = (a - b)/(a + b), out[5] swelling ratio
 *   Sw = A / (P^2 / 4 pi), out[6..8] central second moments Jxx, Jyy, Jxy.
 * Reading: a and b are the semi-axes of the ellipse with the same area second
 * moments, i.e. a : b = sqrt(l1) : sqrt(l2) for the eigenvalues l1 >= l2 of
 * the central second-moment tensor.  Moments are taken about node 0 to limit
 * cancellation, then shifted to the centroid.
 * Pinned: regular polygons (Sw, perimeter), affinely stretched regular
 * polygons (D exactly (a-b)/(a+b)).
 * ------------------------------------------------------------------------- */
void orc_polygon_diag(int nv, const double *x, double out[9])
{
    double ox = x[0], oy = x[1];
    double A2 = 0, P = 0, cxs = 0, cys = 0, ixx = 0, iyy = 0, ixy = 0;
    for (int l = 0; l < nv; l++) {
        int m = (l + 1) % nv;
        double x0 = x[2 * l] - ox, y0 = x[2 * l + 1] - oy;
        double x1 = x[2 * m] - ox, y1 = x[2 * m + 1] - oy;
        double cr = x0 * y1 - x1 * y0;
        A2 += cr;
        P += sqrt((x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0));
        cxs += (x0 + x1) * cr;
        cys += (y0 + y1) * cr;
        ixx += (x0 * x0 + x0 * x1 + x1 * x1) * cr; /* 12 * integral of x^2 dA */
        iyy += (y0 * y0 + y0 * y1 + y1 * y1) * cr;
        ixy += (x0 * y1 + 2 * x0 * y0 + 2 * x1 * y1 + x1 * y0) * cr; /* 24 * integral of xy dA */
    }
    double A = 0.5 * A2;
    double cx = cxs / (6.0 * A), cy = cys / (6.0 * A);
    double jxx = ixx / 12.0 - A * cx * cx;
    double jyy = iyy / 12.0 - A * cy * cy;
    double jxy = ixy / 24.0 - A * cx * cy;
    double tr = 0.5 * (jxx + jyy);
    double disc = sqrt(0.25 * (jxx - jyy) * (jxx - jyy) + jxy * jxy);
    double l1 = tr + disc, l2 = tr - disc;
    double a = sqrt(l1), b = sqrt(l2 > 0 ? l2 : 0);
    out[0] = A;
    out[1] = P;
    out[2] = cx + ox;
    out[3] = cy + oy;
    out[4] = (a - b) / (a + b);
    out[5] = A / (P * P / (4.0 * M_PI));
    out[6] = jxx;
    out[7] = jyy;
    out[8] = jxy;
}

/* ---------------------------------------------------------------------------
 * Simulation state
 * ------------------------------------------------------------------------- */
static void *xcalloc(size_t n, size_t sz)
{
    void *p = calloc(n ? n : 1, sz);
    return p;
}

/* Zou-He known-velocity conditions on the on-node walls y = 0 and y = ny-1
 * (Sec. 2.1, ref. [36]); the wall moves along x at u_w.  Reading: with a body
 * force F at the wall node the tangential momentum target is rho u_w - F_x / 2,
 * so that the force-corrected velocity (Eq. 7) equals the wall speed; the wall
 * normal force is zero in every configuration here.
 * Open channel (periodic_x = 0, Sec. 3.2): Zou-He velocity inlet at x = 0 with
 * the parabolic profile u_x = -u_max((1 - y/(H/2))^2 - 1) = 4 u_max y (H - y) / H^2,
 * u_y = 0, and Zou-He pressure outlet at x = nx-1 with rho = rho_out, u_y = 0
 * (stationary walls and no body force there).  Corner nodes (u = 0): the
 * unknowns opposite a known population take it (bounce-back of the
 * non-equilibrium part), the two remaining "buried" populations share the
 * mass deficit, with the corner density read from the inner diagonal
 * neighbour at the same time level (reading: the paper does not treat the
 * corners). */
static void corner(orc_sim *s, double *f, int x, int y, int nbx, int nby, const int pair[3][2],
                   int b1, int b2)
{
    double *g = f + cid(s, x, y) * 9;
    const double *h = f + cid(s, nbx, nby) * 9;
    double rho = 0.0;
    for (int i = 0; i < 9; i++) rho += h[i];
    for (int p = 0; p < 3; p++) g[pair[p][0]] = g[pair[p][1]];
    double known = 0.0;
    for (int i = 0; i < 9; i++)
        if (i != b1 && i != b2) known += g[i];
    g[b1] = g[b2] = 0.5 * (rho - known);
}

static void zou_he(orc_sim *s, double *f, const double *F)
{
    if (!s->periodic_y) {
        int xa = s->periodic_x ? 0 : 1, xb = s->periodic_x ? s->nx : s->nx - 1;
        for (int x = xa; x < xb; x++) {
            /* bottom wall: f2, f5, f6 unknown */
            double *g = f + cid(s, x, 0) * 9;
            double Fx = F[cid(s, x, 0) * 2];
            double rw = g[0] + g[1] + g[3] + 2.0 * (g[4] + g[7] + g[8]);
            double mx = rw * s->u_bot - 0.5 * Fx;
            g[2] = g[4];
            g[5] = g[7] - 0.5 * (g[1] - g[3]) + 0.5 * mx;
            g[6] = g[8] + 0.5 * (g[1] - g[3]) - 0.5 * mx;
            /* top wall: f4, f7, f8 unknown */
            g = f + cid(s, x, s->ny - 1) * 9;
            Fx = F[cid(s, x, s->ny - 1) * 2];
            rw = g[0] + g[1] + g[3] + 2.0 * (g[2] + g[5] + g[6]);
            mx = rw * s->u_top - 0.5 * Fx;
            g[4] = g[2];
            g[7] = g[5] + 0.5 * (g[1] - g[3]) - 0.5 * mx;
            g[8] = g[6] - 0.5 * (g[1] - g[3]) + 0.5 * mx;
        }
    }
    if (s->periodic_x) return;
    const double H = s->ny - 1;
    for (int y = 1; y < s->ny - 1; y++) {
        /* inlet x = 0: velocity (u_in(y), 0) known, f1, f5, f8 unknown */
        double *g = f + cid(s, 0, y) * 9;
        double ux = 4.0 * s->u_in * y * (H - y) / (H * H);
        double rho = (g[0] + g[2] + g[4] + 2.0 * (g[3] + g[6] + g[7])) / (1.0 - ux);
        g[1] = g[3] + 2.0 / 3.0 * rho * ux;
        g[5] = g[7] - 0.5 * (g[2] - g[4]) + rho * ux / 6.0;
        g[8] = g[6] + 0.5 * (g[2] - g[4]) + rho * ux / 6.0;
        /* outlet x = nx-1: density rho_out known, f3, f6, f7 unknown */
        g = f + cid(s, s->nx - 1, y) * 9;
        double uo = (g[0] + g[2] + g[4] + 2.0 * (g[1] + g[5] + g[8])) / s->rho_out - 1.0;
        g[3] = g[1] - 2.0 / 3.0 * s->rho_out * uo;
        g[7] = g[5] + 0.5 * (g[2] - g[4]) - s->rho_out * uo / 6.0;
        g[6] = g[8] - 0.5 * (g[2] - g[4]) - s->rho_out * uo / 6.0;
    }
    const int nx = s->nx, ny = s->ny;
    static const int bl[3][2] = {{1, 3}, {2, 4}, {5, 7}};
    static const int tl[3][2] = {{1, 3}, {4, 2}, {8, 6}};
    static const int br[3][2] = {{3, 1}, {2, 4}, {6, 8}};
    static const int tr[3][2] = {{3, 1}, {4, 2}, {7, 5}};
    corner(s, f, 0, 0, 1, 1, bl, 6, 8);
    corner(s, f, 0, ny - 1, 1, ny - 2, tl, 5, 7);
    corner(s, f, nx - 1, 0, nx - 2, 1, br, 5, 7);
    corner(s, f, nx - 1, ny - 1, nx - 2, ny - 2, tr, 6, 8);
}

/* Eqs. 6-7: rho = sum f, rho u = sum f e + F/2 (reading: the half term is the
 * force density, as in Guo's scheme; the printed "F_i/2" is garbled). */
static void moments(orc_sim *s)
{
#pragma omp parallel for schedule(static)
    for (int x = 0; x < s->nx; x++)
        for (int y = 0; y < s->ny; y++) {
            size_t c = cid(s, x, y);
            const double *g = s->f + c * 9;
            double r = 0, jx = 0, jy = 0;
            for (int i = 0; i < 9; i++) {
                r += g[i];
                jx += g[i] * EX[i];
                jy += g[i] * EY[i];
            }
            s->rho[c] = r;
            s->ux[c] = (jx + 0.5 * s->F[c * 2]) / r;
            s->uy[c] = (jy + 0.5 * s->F[c * 2 + 1]) / r;
        }
}

/* Eq. 4 with Eq. 5: one BGK collision with forcing F at every node, then
 * streaming f_i(x + e_i) <- post-collision f_i(x); periodic in x (and in y for
 * a fully periodic box), Zou-He on the walls.  The velocity inside f^eq and the
 * forcing term is the force-corrected one of Eq. 7 with the same F. */
static void collide_stream(orc_sim *s)
{
    const double *F = s->F;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < s->nx; x++)
        for (int y = 0; y < s->ny; y++) {
            size_t c = cid(s, x, y);
            const double *g = s->f + c * 9;
            double r = 0, jx = 0, jy = 0;
            for (int i = 0; i < 9; i++) {
                r += g[i];
                jx += g[i] * EX[i];
                jy += g[i] * EY[i];
            }
            double ux = (jx + 0.5 * F[c * 2]) / r, uy = (jy + 0.5 * F[c * 2 + 1]) / r;
            double feq[9], src[9];
            orc_equilibrium(r, ux, uy, feq);
            orc_forcing(s->tau, ux, uy, F[c * 2], F[c * 2 + 1], src);
            for (int i = 0; i < 9; i++) {
                double post = g[i] - (g[i] - feq[i]) / s->tau + src[i];
                int xd = x + EX[i], yd = y + EY[i];
                if (s->periodic_x) xd = wrap(xd, s->nx);
                else if (xd < 0 || xd >= s->nx) continue;
                if (s->periodic_y) yd = wrap(yd, s->ny);
                else if (yd < 0 || yd >= s->ny) continue;
                s->ftmp[cid(s, xd, yd) * 9 + i] = post;
            }
        }
    zou_he(s, s->ftmp, F);
    double *t = s->f;
    s->f = s->ftmp;
    s->ftmp = t;
}

/* lattice field lookup at an unwrapped support node; flags supports that reach
 * a wall row (the MLS support must lie in the fluid interior) */
static int field_index(orc_sim *s, int cx, int cy, size_t *out)
{
    int x = wrap(cx, s->nx), y = cy;
    if (!s->periodic_x && (cx < 1 || cx > s->nx - 2)) {
        s->status |= ORC_E_WALL;
        return 0;
    }
    if (s->periodic_y) y = wrap(cy, s->ny);
    else if (cy < 1 || cy > s->ny - 2) {
        s->status |= ORC_E_WALL;
        return 0;
    }
    *out = cid(s, x, y);
    return 1;
}

/* Eq. 8: U(x) = sum_k phi_k u_k over the MLS support of x */
static void interpolate_u(orc_sim *s, double xm, double ym, double *U)
{
    int cx[9], cy[9];
    double phi[9], dx[9], dy[9];
    orc_mls(xm, ym, cx, cy, phi, dx, dy);
    U[0] = U[1] = 0.0;
    for (int k = 0; k < 9; k++) {
        size_t c;
        if (!field_index(s, cx[k], cy[k], &c)) continue;
        U[0] += phi[k] * s->ux[c];
        U[1] += phi[k] * s->uy[c];
    }
}

/* Dynamic step 3 / Kinematic step iii: f_ib(x_k) += c phi_k(x) F */
static void spread(orc_sim *s, double xm, double ym, double c, double Fx, double Fy)
{
    int cx[9], cy[9];
    double phi[9], dx[9], dy[9];
    orc_mls(xm, ym, cx, cy, phi, dx, dy);
    for (int k = 0; k < 9; k++) {
        size_t cc;
        if (!field_index(s, cx[k], cy[k], &cc)) continue;
        s->fib[cc * 2] += c * phi[k] * Fx;
        s->fib[cc * 2 + 1] += c * phi[k] * Fy;
    }
}

/* MLS pressure p = c_s^2 rho and velocity gradient G[a][b] = d u_a / d x_b at a probe */
static void probe_state(orc_sim *s, double xp, double yp, double *p, double G[2][2])
{
    int cx[9], cy[9];
    double phi[9], dx[9], dy[9];
    orc_mls(xp, yp, cx, cy, phi, dx, dy);
    double rho = 0;
    G[0][0] = G[0][1] = G[1][0] = G[1][1] = 0;
    for (int k = 0; k < 9; k++) {
        size_t c;
        if (!field_index(s, cx[k], cy[k], &c)) continue;
        rho += phi[k] * s->rho[c];
        G[0][0] += dx[k] * s->ux[c];
        G[0][1] += dy[k] * s->ux[c];
        G[1][0] += dx[k] * s->uy[c];
        G[1][1] += dy[k] * s->uy[c];
    }
    *p = CS2 * rho;
}

/* ---------------------------------------------------------------------------
 * Eqs. 15-16: hydrodynamic element forces from probes at the element centroid
 * +- 1.2 dx along n+ (Sec. 2.2.2), using the current lattice moments:
 *   F_p = -(p+ - p-) n+ l,  F_tau = (tau+ - tau-) . n+ l,
 *   tau = rho_ref nu (grad u + grad u^T)  (reading: rho_ref = 1, pressure
 *   c_s^2 times the interpolated density).
 * Reading: the element force goes half to each end node.
 * Pinned: a linear pressure field and a piecewise-linear shear field give the
 * closed-form element forces.
 * ------------------------------------------------------------------------- */
static void external_forces(orc_sim *s, int nv, const double *x, double *fext)
{
    memset(fext, 0, sizeof(double) * 2 * nv);
    for (int l = 0; l < nv; l++) {
        int v1 = l, v2 = (l + 1) % nv;
        double tx = x[2 * v2] - x[2 * v1], ty = x[2 * v2 + 1] - x[2 * v1 + 1];
        double len = sqrt(tx * tx + ty * ty);
        double npx = ty / len, npy = -tx / len;
        double xc = 0.5 * (x[2 * v1] + x[2 * v2]), yc = 0.5 * (x[2 * v1 + 1] + x[2 * v2 + 1]);
        double pp, pm, Gp[2][2], Gm[2][2];
        probe_state(s, xc + PROBE_LEN * npx, yc + PROBE_LEN * npy, &pp, Gp);
        probe_state(s, xc - PROBE_LEN * npx, yc - PROBE_LEN * npy, &pm, Gm);
        double tp[2][2], tm[2][2];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                tp[a][b] = 1.0 * s->nu * (Gp[a][b] + Gp[b][a]);
                tm[a][b] = 1.0 * s->nu * (Gm[a][b] + Gm[b][a]);
            }
        double Fx = -(pp - pm) * npx * len + ((tp[0][0] - tm[0][0]) * npx + (tp[0][1] - tm[0][1]) * npy) * len;
        double Fy = -(pp - pm) * npy * len + ((tp[1][0] - tm[1][0]) * npx + (tp[1][1] - tm[1][1]) * npy) * len;
        fext[2 * v1] += 0.5 * Fx;
        fext[2 * v1 + 1] += 0.5 * Fy;
        fext[2 * v2] += 0.5 * Fx;
        fext[2 * v2 + 1] += 0.5 * Fy;
    }
}

/* ---------------------------------------------------------------------------
 * Public API
 * ------------------------------------------------------------------------- */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* init_profile: 0 rest, 1 linear Couette between the wall speeds, 2 analytic
 * body-force Poiseuille u = g/(2 nu) y (H - y) with H = ny - 1, 3 uniform (u0x, u0y).
 * f^0 = f^eq(1, u_init); the wall condition is then applied with F = g and the
 * moments are taken with half of F^{-1} = g. */
orc_sim *orc_create(int nx, int ny, double tau, int periodic_y, double u_bot, double u_top,
                    double gx, double gy, int init_profile, double u0x, double u0y, int periodic_x,
                    double u_in, double rho_out)
{
    orc_sim *s = (orc_sim *)xcalloc(1, sizeof(orc_sim));
    s->nx = nx;
    s->ny = ny;
    s->periodic_y = periodic_y;
    s->periodic_x = periodic_x;
    s->u_in = u_in;
    s->rho_out = rho_out;
    s->tau = tau;
    s->nu = CS2 * (tau - 0.5); /* Sec. 2.1, dt = 1 */
    s->u_bot = u_bot;
    s->u_top = u_top;
    s->gx = gx;
    s->gy = gy;
    size_t n = (size_t)nx * ny;
    s->f = (double *)xcalloc(n * 9, sizeof(double));
    s->ftmp = (double *)xcalloc(n * 9, sizeof(double));
    s->F = (double *)xcalloc(n * 2, sizeof(double));
    s->fib = (double *)xcalloc(n * 2, sizeof(double));
    s->rho = (double *)xcalloc(n, sizeof(double));
    s->ux = (double *)xcalloc(n, sizeof(double));
    s->uy = (double *)xcalloc(n, sizeof(double));
    s->mode = -1;
    double H = ny - 1;
    for (int x = 0; x < nx; x++)
        for (int y = 0; y < ny; y++) {
            double ux = 0, uy = 0;
            if (init_profile == 1) ux = u_bot + (u_top - u_bot) * y / H;
            else if (init_profile == 2) ux = gx / (2.0 * s->nu) * y * (H - y);
            else if (init_profile == 3) { ux = u0x; uy = u0y; }
            else if (init_profile == 4) ux = 4.0 * u_in * y * (H - y) / (H * H);
            orc_equilibrium(1.0, ux, uy, s->f + cid(s, x, y) * 9);
            s->F[cid(s, x, y) * 2] = gx;
            s->F[cid(s, x, y) * 2 + 1] = gy;
        }
    zou_he(s, s->f, s->F);
    moments(s);
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int c = 0; c < s->ncap; c++) {
        orc_capsule *k = &s->caps[c];
        free(k->x); free(k->xm1); free(k->uv); free(k->l0); free(k->theta0);
        free(k->ks); free(k->ftot); free(k->fext); free(k->fc); free(k->r0);
    }
    free(s->caps);
    free(s->f); free(s->ftmp); free(s->F); free(s->fib);
    free(s->rho); free(s->ux); free(s->uy);
    free(s);
}

/* Adds a capsule whose given node positions are its stress-free shape:
 * l0, theta0, A0 and P0 are taken from them (Sec. 2.2.1); the mass is spread
 * evenly over the nodes, m_v = mass / nv (Sec. 2.3.2).  ks holds n_ks = 1 or
 * nv per-element values. */
int orc_add_capsule(orc_sim *s, int nv, const double *nodes, const double *ks, int n_ks,
                    double kb, double ka, double mass)
{
    if (s->ncap == s->capcap) {
        s->capcap = s->capcap ? 2 * s->capcap : 8;
        s->caps = (orc_capsule *)realloc(s->caps, sizeof(orc_capsule) * s->capcap);
    }
    orc_capsule *k = &s->caps[s->ncap];
    memset(k, 0, sizeof(*k));
    k->nv = nv;
    k->x = (double *)xcalloc(2 * nv, sizeof(double));
    k->xm1 = (double *)xcalloc(2 * nv, sizeof(double));
    k->uv = (double *)xcalloc(2 * nv, sizeof(double));
    k->l0 = (double *)xcalloc(nv, sizeof(double));
    k->theta0 = (double *)xcalloc(nv, sizeof(double));
    k->ks = (double *)xcalloc(nv, sizeof(double));
    k->ftot = (double *)xcalloc(2 * nv, sizeof(double));
    k->fext = (double *)xcalloc(2 * nv, sizeof(double));
    k->fc = (double *)xcalloc(2 * nv, sizeof(double));
    memcpy(k->x, nodes, sizeof(double) * 2 * nv);
    double P = 0;
    for (int l = 0; l < nv; l++) {
        int m = (l + 1) % nv;
        double dx = nodes[2 * m] - nodes[2 * l], dy = nodes[2 * m + 1] - nodes[2 * l + 1];
        k->l0[l] = sqrt(dx * dx + dy * dy);
        P += k->l0[l];
        k->theta0[l] = turning_angle(nv, nodes, l);
        k->ks[l] = n_ks == 1 ? ks[0] : ks[l];
    }
    k->kb = kb;
    k->ka = ka;
    k->mass = mass;
    k->mv = mass / nv;
    k->A0 = polygon_area(nv, nodes);
    k->P0 = P;
    k->primed = 0;
    return s->ncap++;
}

/* Eq. 27: repulsion between the vertices of different capsules (Sec. 3.4).
 * Vertex i of capsule a, at distance d < cutoff from vertex j of capsule b,
 * receives (1e-4 / (8 sqrt 2)) sqrt(dx / d^5) along its inward normal n-,
 * summed over all such j; dx = 1.  Readings: the cutoff is not printed (the
 * caller sets it, 2 dx by default in the workloads); the vertex normal is the
 * normalized sum of the outward normals of its two elements.  Distances take
 * the nearest periodic image.  Evaluated at the current positions of every
 * capsule, before any of them moves. */
static void contact_forces(orc_sim *s)
{
    const double C = 1e-4 / (8.0 * sqrt(2.0));
    for (int a = 0; a < s->ncap; a++)
        memset(s->caps[a].fc, 0, sizeof(double) * 2 * s->caps[a].nv);
    if (!(s->contact_cutoff > 0.0)) return;
    for (int a = 0; a < s->ncap; a++) {
        orc_capsule *ka = &s->caps[a];
        int nv = ka->nv;
        for (int i = 0; i < nv; i++) {
            int il = (i + nv - 1) % nv, ir = (i + 1) % nv;
            double ax = ka->x[2 * i] - ka->x[2 * il], ay = ka->x[2 * i + 1] - ka->x[2 * il + 1];
            double bx = ka->x[2 * ir] - ka->x[2 * i], by = ka->x[2 * ir + 1] - ka->x[2 * i + 1];
            double la = hypot(ax, ay), lb = hypot(bx, by);
            /* outward element normals (t_y, -t_x)/|t| of elements i-1 and i */
            double nx = ay / la + by / lb, ny = -ax / la - bx / lb;
            double nn = hypot(nx, ny);
            double inx = -nx / nn, iny = -ny / nn;
            for (int b = 0; b < s->ncap; b++) {
                if (b == a) continue;
                orc_capsule *kb = &s->caps[b];
                for (int j = 0; j < kb->nv; j++) {
                    double dx = kb->x[2 * j] - ka->x[2 * i];
                    double dy = kb->x[2 * j + 1] - ka->x[2 * i + 1];
                    if (s->periodic_x) dx -= s->nx * nearbyint(dx / s->nx);
                    if (s->periodic_y) dy -= s->ny * nearbyint(dy / s->ny);
                    double d = hypot(dx, dy);
                    if (d < s->contact_cutoff && d > 0.0) {
                        double mag = C * sqrt(1.0 / (d * d * d * d * d));
                        ka->fc[2 * i] += mag * inx;
                        ka->fc[2 * i + 1] += mag * iny;
                    }
                }
            }
        }
    }
}

/* Adds a rigid particle (Sec. 2.3.1) with the given node outline (counter-
 * clockwise), total mass m and moment of inertia I about the area centroid.
 * It moves with the Dynamic scheme only: direct forcing towards the rigid-body
 * velocity of each node, force and torque from the outer probes (Eqs. 17-18),
 * velocities by Eqs. 19-20. */
int orc_add_rigid(orc_sim *s, int nv, const double *nodes, double mass, double inertia)
{
    double ks = 0.0;
    int c = orc_add_capsule(s, nv, nodes, &ks, 1, 0.0, 0.0, mass);
    orc_capsule *k = &s->caps[c];
    k->rigid = 1;
    k->I = inertia;
    double A2 = 0, cx = 0, cy = 0;
    for (int l = 0; l < nv; l++) {
        int m = (l + 1) % nv;
        double cr = nodes[2 * l] * nodes[2 * m + 1] - nodes[2 * m] * nodes[2 * l + 1];
        A2 += cr;
        cx += (nodes[2 * l] + nodes[2 * m]) * cr;
        cy += (nodes[2 * l + 1] + nodes[2 * m + 1]) * cr;
    }
    k->X[0] = cx / (3.0 * A2);
    k->X[1] = cy / (3.0 * A2);
    k->theta = 0.0;
    k->r0 = (double *)xcalloc(2 * nv, sizeof(double));
    for (int v = 0; v < nv; v++) {
        k->r0[2 * v] = nodes[2 * v] - k->X[0];
        k->r0[2 * v + 1] = nodes[2 * v + 1] - k->X[1];
    }
    return c;
}

void orc_get_rigid(const orc_sim *s, int c, double out[10])
{
    const orc_capsule *k = &s->caps[c];
    out[0] = k->X[0]; out[1] = k->X[1]; out[2] = k->theta;
    out[3] = k->u[0]; out[4] = k->u[1]; out[5] = k->w;
    out[6] = k->Ftot[0]; out[7] = k->Ftot[1]; out[8] = k->Mtot; out[9] = k->rigid;
}

/* Eqs. 17-18: force and torque of the fluid on a rigid particle from the
 * stresses at the outer probes x_c + 1.2 n+ of every element (pressure as the
 * deviation c_s^2 (rho - 1): a uniform pressure gives no net force or torque
 * on a closed polygon).  Torque about the centroid X with the element
 * centroid as lever point.  The contact forces of Eq. 27 on its nodes add to
 * both. */
static void rigid_loads(orc_sim *s, orc_capsule *k)
{
    int nv = k->nv;
    const double *x = k->x;
    k->Ftot[0] = k->Ftot[1] = k->Mtot = 0.0;
    for (int l = 0; l < nv; l++) {
        int v1 = l, v2 = (l + 1) % nv;
        double tx = x[2 * v2] - x[2 * v1], ty = x[2 * v2 + 1] - x[2 * v1 + 1];
        double len = sqrt(tx * tx + ty * ty);
        double npx = ty / len, npy = -tx / len;
        double xc = 0.5 * (x[2 * v1] + x[2 * v2]), yc = 0.5 * (x[2 * v1 + 1] + x[2 * v2 + 1]);
        double pp, Gp[2][2];
        probe_state(s, xc + PROBE_LEN * npx, yc + PROBE_LEN * npy, &pp, Gp);
        pp -= CS2;
        double t00 = s->nu * 2.0 * Gp[0][0], t11 = s->nu * 2.0 * Gp[1][1];
        double t01 = s->nu * (Gp[0][1] + Gp[1][0]);
        double fx = (t00 * npx + t01 * npy - pp * npx) * len;
        double fy = (t01 * npx + t11 * npy - pp * npy) * len;
        k->Ftot[0] += fx;
        k->Ftot[1] += fy;
        k->Mtot += (xc - k->X[0]) * fy - (yc - k->X[1]) * fx;
    }
    /* contact forces on the nodes (Eq. 27) act on the body as a whole */
    for (int v = 0; v < nv; v++) {
        k->Ftot[0] += k->fc[2 * v];
        k->Ftot[1] += k->fc[2 * v + 1];
        k->Mtot += (x[2 * v] - k->X[0]) * k->fc[2 * v + 1] - (x[2 * v + 1] - k->X[1]) * k->fc[2 * v];
    }
}

/* Eqs. 19-20 and the rigid-body kinematics: new velocities from the
 * accelerations F/m and M/I, then (reading: the paper prints no position
 * update) X^{n+1} = X^n + u^{n+1} dt, theta^{n+1} = theta^n + w^{n+1} dt and
 * x_v = X + R(theta) r0_v.  uv holds the nodes' rigid-body velocities. */
static void rigid_update(orc_capsule *k)
{
    double ax = k->Ftot[0] / k->mass, ay = k->Ftot[1] / k->mass, aw = k->Mtot / k->I;
    double ux = 2.0 / 3.0 * (2.0 * k->u[0] - 0.5 * k->um1[0] + ax * 1.0);
    double uy = 2.0 / 3.0 * (2.0 * k->u[1] - 0.5 * k->um1[1] + ay * 1.0);
    double w = 2.0 / 3.0 * (2.0 * k->w - 0.5 * k->wm1 + aw * 1.0);
    k->um1[0] = k->u[0]; k->um1[1] = k->u[1]; k->wm1 = k->w;
    k->u[0] = ux; k->u[1] = uy; k->w = w;
    k->X[0] += ux * 1.0;
    k->X[1] += uy * 1.0;
    k->theta += w * 1.0;
    double c = cos(k->theta), sn = sin(k->theta);
    memcpy(k->xm1, k->x, sizeof(double) * 2 * k->nv);
    for (int v = 0; v < k->nv; v++) {
        double rx = c * k->r0[2 * v] - sn * k->r0[2 * v + 1];
        double ry = sn * k->r0[2 * v] + c * k->r0[2 * v + 1];
        k->x[2 * v] = k->X[0] + rx;
        k->x[2 * v + 1] = k->X[1] + ry;
        k->uv[2 * v] = ux - w * ry;
        k->uv[2 * v + 1] = uy + w * rx;
    }
}

void orc_set_contact(orc_sim *s, double cutoff) { s->contact_cutoff = cutoff > 0.0 ? cutoff : 0.0; }

void orc_get_contact(const orc_sim *s, int c, double *fc)
{
    memcpy(fc, s->caps[c].fc, sizeof(double) * 2 * s->caps[c].nv);
}

/* Start-up (reading: the paper gives no history at n = 0): the node velocity
 * is the interpolated fluid velocity, u_v^0 = U(x^0), and x^{-1} = x^0 - U(x^0),
 * so the first direct-forcing term vanishes and uniform motion is exact. */
static void prime(orc_sim *s, orc_capsule *k)
{
    if (k->rigid) {
        /* reading: u^0 = u^{-1} = mean node velocity of the fluid, w^0 = w^{-1}
         * = the least-squares rigid rotation of the interpolated velocities */
        double su[2] = {0, 0}, num = 0, den = 0;
        for (int v = 0; v < k->nv; v++) {
            double U[2];
            interpolate_u(s, k->x[2 * v], k->x[2 * v + 1], U);
            double rx = k->x[2 * v] - k->X[0], ry = k->x[2 * v + 1] - k->X[1];
            su[0] += U[0];
            su[1] += U[1];
            num += rx * U[1] - ry * U[0];
            den += rx * rx + ry * ry;
        }
        k->u[0] = k->um1[0] = su[0] / k->nv;
        k->u[1] = k->um1[1] = su[1] / k->nv;
        k->w = k->wm1 = num / den;
        for (int v = 0; v < k->nv; v++) {
            double rx = k->x[2 * v] - k->X[0], ry = k->x[2 * v + 1] - k->X[1];
            k->uv[2 * v] = k->u[0] - k->w * ry;
            k->uv[2 * v + 1] = k->u[1] + k->w * rx;
            k->xm1[2 * v] = k->x[2 * v] - k->uv[2 * v];
            k->xm1[2 * v + 1] = k->x[2 * v + 1] - k->uv[2 * v + 1];
        }
        k->primed = 1;
        return;
    }
    for (int v = 0; v < k->nv; v++) {
        double U[2];
        interpolate_u(s, k->x[2 * v], k->x[2 * v + 1], U);
        k->uv[2 * v] = U[0];
        k->uv[2 * v + 1] = U[1];
        k->xm1[2 * v] = k->x[2 * v] - U[0];
        k->xm1[2 * v + 1] = k->x[2 * v + 1] - U[1];
    }
    k->primed = 1;
}

static void check_finite(orc_sim *s)
{
    for (int c = 0; c < s->ncap; c++)
        for (int j = 0; j < 2 * s->caps[c].nv; j++)
            if (!isfinite(s->caps[c].x[j])) s->status |= ORC_E_NONFINITE;
}

/* One time step of the Dynamic IB scheme (Sec. 2.3.2, steps 1-8). */
static void step_dynamic(orc_sim *s)
{
    size_t n = (size_t)s->nx * s->ny;
    memset(s->fib, 0, sizeof(double) * 2 * n);
    /* steps 1-3: forcing F_v = (u_v^n - U(x_v^n)) / dt at each node, with U
     * interpolated (Eq. 8) from the current moments u^n, spread to the
     * lattice with c_v = arc length carried by the node (reading: "total force
     * conservation" with F_v an acceleration gives the node's share of the
     * membrane, (l_{v-1} + l_v)/2, over dx^2 = 1).  Reading: markers are the
     * nodes (vertices) for interpolation, forcing and spreading. */
    for (int c = 0; c < s->ncap; c++) {
        orc_capsule *k = &s->caps[c];
        int nv = k->nv;
        for (int v = 0; v < nv; v++) {
            double U[2];
            interpolate_u(s, k->x[2 * v], k->x[2 * v + 1], U);
            double Fx = k->uv[2 * v] - U[0], Fy = k->uv[2 * v + 1] - U[1];
            int vl = (v + nv - 1) % nv, vr = (v + 1) % nv;
            double ll = hypot(k->x[2 * v] - k->x[2 * vl], k->x[2 * v + 1] - k->x[2 * vl + 1]);
            double lr = hypot(k->x[2 * vr] - k->x[2 * v], k->x[2 * vr + 1] - k->x[2 * v + 1]);
            spread(s, k->x[2 * v], k->x[2 * v + 1], 0.5 * (ll + lr), Fx, Fy);
        }
    }
    /* steps 4-5: forcing term (Eq. 5) with F^n = f_ib + g, BGK update (Eq. 4) */
    for (size_t c = 0; c < n; c++) {
        s->F[c * 2] = s->fib[c * 2] + s->gx;
        s->F[c * 2 + 1] = s->fib[c * 2 + 1] + s->gy;
    }
    collide_stream(s);
    /* step 6: moments of f^{n+1} (Eqs. 6-7) with half of the force just applied */
    moments(s);
    /* steps 7-8: total nodal force at x^n (internal Eqs. 11, 13, 14 plus
     * hydrodynamic Eqs. 15-16 from the new moments), Verlet position update
     * (Eq. 23) with the tentative velocity interpolated from u^{n+1}
     * (reading), BDF2 node velocity (Eq. 24).  The contact force (Eq. 27) of
     * x^n joins the total force. */
    contact_forces(s);
    for (int c = 0; c < s->ncap; c++) {
        orc_capsule *k = &s->caps[c];
        int nv = k->nv;
        if (k->rigid) {  /* Sec. 2.3.1 */
            rigid_loads(s, k);
            rigid_update(k);
            continue;
        }
        double *fs = (double *)xcalloc(2 * nv, sizeof(double));
        double *fb = (double *)xcalloc(2 * nv, sizeof(double));
        double *fa = (double *)xcalloc(2 * nv, sizeof(double));
        orc_internal_forces(nv, k->x, k->l0, k->theta0, k->ks, k->kb, k->ka, k->A0, fs, fb, fa);
        external_forces(s, nv, k->x, k->fext);
        double *xn = (double *)xcalloc(2 * nv, sizeof(double));
        for (int v = 0; v < nv; v++) {
            double U[2];
            interpolate_u(s, k->x[2 * v], k->x[2 * v + 1], U);
            for (int d = 0; d < 2; d++) {
                int j = 2 * v + d;
                k->ftot[j] = fs[j] + fb[j] + fa[j] + k->fext[j] + k->fc[j];
                xn[j] = k->x[j] + U[d] * 1.0 + 0.5 * k->ftot[j] / k->mv * 1.0;
                k->uv[j] = (1.5 * xn[j] - 2.0 * k->x[j] + 0.5 * k->xm1[j]) / 1.0;
            }
        }
        memcpy(k->xm1, k->x, sizeof(double) * 2 * nv);
        memcpy(k->x, xn, sizeof(double) * 2 * nv);
        free(fs); free(fb); free(fa); free(xn);
    }
}

/* One time step of the Kinematic IB scheme (Sec. 2.4, steps i-viii). */
static void step_kinematic(orc_sim *s)
{
    size_t n = (size_t)s->nx * s->ny;
    memset(s->fib, 0, sizeof(double) * 2 * n);
    /* i-iii: internal forces (and the contact force of Eq. 27 at x^n), spread
     * with c_v = 1 (reading: F_v is a nodal force, so c_v = 1 / dx^2) */
    contact_forces(s);
    for (int c = 0; c < s->ncap; c++) {
        orc_capsule *k = &s->caps[c];
        int nv = k->nv;
        double *fs = (double *)xcalloc(2 * nv, sizeof(double));
        double *fb = (double *)xcalloc(2 * nv, sizeof(double));
        double *fa = (double *)xcalloc(2 * nv, sizeof(double));
        orc_internal_forces(nv, k->x, k->l0, k->theta0, k->ks, k->kb, k->ka, k->A0, fs, fb, fa);
        for (int v = 0; v < nv; v++) {
            k->ftot[2 * v] = fs[2 * v] + fb[2 * v] + fa[2 * v] + k->fc[2 * v];
            k->ftot[2 * v + 1] = fs[2 * v + 1] + fb[2 * v + 1] + fa[2 * v + 1] + k->fc[2 * v + 1];
            spread(s, k->x[2 * v], k->x[2 * v + 1], 1.0, k->ftot[2 * v], k->ftot[2 * v + 1]);
        }
        free(fs); free(fb); free(fa);
    }
    /* iv-v (reading: the f_ib of step iii of this same step) */
    for (size_t c = 0; c < n; c++) {
        s->F[c * 2] = s->fib[c * 2] + s->gx;
        s->F[c * 2 + 1] = s->fib[c * 2 + 1] + s->gy;
    }
    collide_stream(s);
    /* vi */
    moments(s);
    /* vii-viii: x^{n+1} = 2/3 (2 x^n - x^{n-1}/2 + xdot dt), Eq. 25 */
    for (int c = 0; c < s->ncap; c++) {
        orc_capsule *k = &s->caps[c];
        int nv = k->nv;
        double *xn = (double *)xcalloc(2 * nv, sizeof(double));
        for (int v = 0; v < nv; v++) {
            double U[2];
            interpolate_u(s, k->x[2 * v], k->x[2 * v + 1], U);
            for (int d = 0; d < 2; d++) {
                int j = 2 * v + d;
                xn[j] = 2.0 / 3.0 * (2.0 * k->x[j] - 0.5 * k->xm1[j] + U[d] * 1.0);
            }
        }
        memcpy(k->xm1, k->x, sizeof(double) * 2 * nv);
        memcpy(k->x, xn, sizeof(double) * 2 * nv);
        free(xn);
    }
}

/* mode: 0 Kinematic, 1 Dynamic; fixed for the life of the simulation.
 * Returns 0, or -4 if the mode changes after the first step. */
int orc_step(orc_sim *s, int nsteps, int mode)
{
    if (s->mode >= 0 && s->mode != mode) return -4;
    for (int c = 0; c < s->ncap; c++)
        if (s->caps[c].rigid && mode != ORC_DYNAMIC) return -5;  /* rigid: Dynamic only */
    s->mode = mode;
    for (int t = 0; t < nsteps; t++) {
        for (int c = 0; c < s->ncap; c++)
            if (!s->caps[c].primed) prime(s, &s->caps[c]);
        if (mode == ORC_DYNAMIC) step_dynamic(s);
        else step_kinematic(s);
        s->steps++;
        check_finite(s);
    }
    return 0;
}

/* ---- accessors (public layout [component][y][x]) ---- */
int orc_status(const orc_sim *s) { return s->status; }
long orc_steps(const orc_sim *s) { return s->steps; }
int orc_num_capsules(const orc_sim *s) { return s->ncap; }
int orc_capsule_nodes(const orc_sim *s, int c) { return s->caps[c].nv; }

void orc_get_pops(const orc_sim *s, double *out)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int i = 0; i < 9; i++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++)
                out[i * plane + (size_t)y * s->nx + x] = s->f[cid(s, x, y) * 9 + i];
}

/* Replaces f^n; the wall condition is re-applied with the stored force and the
 * moments are recomputed. */
void orc_set_pops(orc_sim *s, const double *in)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int i = 0; i < 9; i++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++)
                s->f[cid(s, x, y) * 9 + i] = in[i * plane + (size_t)y * s->nx + x];
    zou_he(s, s->f, s->F);
    moments(s);
}

/* out: rho, ux, uy planes [3][ny][nx] (moments with half of the last force) */
void orc_get_moments(const orc_sim *s, double *out)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            size_t o = (size_t)y * s->nx + x;
            out[o] = s->rho[cid(s, x, y)];
            out[plane + o] = s->ux[cid(s, x, y)];
            out[2 * plane + o] = s->uy[cid(s, x, y)];
        }
}

/* F^{n-1}: total force of the last collision, [2][ny][nx] */
void orc_get_force(const orc_sim *s, double *out)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            out[(size_t)y * s->nx + x] = s->F[cid(s, x, y) * 2];
            out[plane + (size_t)y * s->nx + x] = s->F[cid(s, x, y) * 2 + 1];
        }
}

/* Sets F^{n-1} (used for the half-force in the moments) and recomputes them. */
void orc_set_force(orc_sim *s, const double *in)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            s->F[cid(s, x, y) * 2] = in[(size_t)y * s->nx + x];
            s->F[cid(s, x, y) * 2 + 1] = in[plane + (size_t)y * s->nx + x];
        }
    moments(s);
}

/* Overwrites the moment fields (test hook for the hydrodynamic-force pins);
 * in: rho, ux, uy planes [3][ny][nx]. */
void orc_set_moments(orc_sim *s, const double *in)
{
    size_t plane = (size_t)s->nx * s->ny;
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            size_t o = (size_t)y * s->nx + x;
            s->rho[cid(s, x, y)] = in[o];
            s->ux[cid(s, x, y)] = in[plane + o];
            s->uy[cid(s, x, y)] = in[2 * plane + o];
        }
}

/* x^n, x^{n-1}, u_v^n of capsule c, each [nv][2] */
void orc_get_capsule(const orc_sim *s, int c, double *x, double *xm1, double *uv)
{
    const orc_capsule *k = &s->caps[c];
    if (x) memcpy(x, k->x, sizeof(double) * 2 * k->nv);
    if (xm1) memcpy(xm1, k->xm1, sizeof(double) * 2 * k->nv);
    if (uv) memcpy(uv, k->uv, sizeof(double) * 2 * k->nv);
}

/* Sets the node history of capsule c and marks it started. */
void orc_set_capsule(orc_sim *s, int c, const double *x, const double *xm1, const double *uv)
{
    orc_capsule *k = &s->caps[c];
    memcpy(k->x, x, sizeof(double) * 2 * k->nv);
    memcpy(k->xm1, xm1, sizeof(double) * 2 * k->nv);
    memcpy(k->uv, uv, sizeof(double) * 2 * k->nv);
    k->primed = 1;
}

/* last total (Dynamic) / internal (Kinematic) nodal force and hydrodynamic force */
void orc_get_capsule_forces(const orc_sim *s, int c, double *ftot, double *fext)
{
    const orc_capsule *k = &s->caps[c];
    if (ftot) memcpy(ftot, k->ftot, sizeof(double) * 2 * k->nv);
    if (fext) memcpy(fext, k->fext, sizeof(double) * 2 * k->nv);
}

/* out[0..8] as orc_polygon_diag, out[9] perimeter change (P - P0)/P0,
 * out[10] A/A0 - 1, out[11] A0, out[12] P0 */
void orc_get_diag(const orc_sim *s, int c, double out[13])
{
    const orc_capsule *k = &s->caps[c];
    orc_polygon_diag(k->nv, k->x, out);
    out[9] = (out[1] - k->P0) / k->P0;
    out[10] = out[0] / k->A0 - 1.0;
    out[11] = k->A0;
    out[12] = k->P0;
}

/* Hydrodynamic nodal forces (Eqs. 15-16) of an arbitrary polygon against the
 * current moment fields (test hook). */
void orc_external_forces(orc_sim *s, int nv, const double *x, double *fext)
{
    external_forces(s, nv, x, fext);
}

/* MLS interpolation of the current velocity at n points (test hook); xy [n][2] */
void orc_interpolate(orc_sim *s, int n, const double *xy, double *U)
{
    for (int j = 0; j < n; j++) interpolate_u(s, xy[2 * j], xy[2 * j + 1], U + 2 * j);
}

/* Spreads n point forces with weights c into a zeroed f_ib and returns it
 * [2][ny][nx] (test hook for the spreading pins). */
void orc_spread(orc_sim *s, int n, const double *xy, const double *c, const double *F,
                double *out)
{
    size_t plane = (size_t)s->nx * s->ny;
    memset(s->fib, 0, sizeof(double) * 2 * plane);
    for (int j = 0; j < n; j++) spread(s, xy[2 * j], xy[2 * j + 1], c[j], F[2 * j], F[2 * j + 1]);
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            out[(size_t)y * s->nx + x] = s->fib[cid(s, x, y) * 2];
            out[plane + (size_t)y * s->nx + x] = s->fib[cid(s, x, y) * 2 + 1];
        }
}
