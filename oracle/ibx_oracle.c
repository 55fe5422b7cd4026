/*
 * ibx_oracle.c -- plain, slow, FP64 reference of the multidirect-forcing
 * immersed-boundary (IB) loop of Li et al., "An open-source, adaptive solver
 * for particle-resolved simulations with both subcycling and non-subcycling
 * methods" (arXiv 2408.14140).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded solely by the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark.  It shares no code, header or table with the GPU library.
 *
 * Everything is FP64 over a global cell-centred grid u[c][z][y][x] (x
 * fastest) of n[0] x n[1] x n[2] cells of size h starting at lo.  Loops
 * follow the paper's equations term by term; nothing is blocked, fused or
 * reordered.  The default build (liboracle.so) is single-threaded.  The same
 * source compiled with OpenMP (liboracle_omp.so) splits the loops of
 * Algorithm 1 without changing any sum's order: interpolation and the
 * velocity correction are independent per marker and per cell; spreading
 * gives each thread a slab of z planes, and every thread visits all markers
 * in index order and adds only into its own planes, so each cell receives
 * its contributions in the serial order.  Both builds give identical bits.
 *
 * Readings of points the paper leaves open (kept identical in the GPU library
 * by its own code):
 *   - delta kernels: the 3-point kernel of Roma, Peskin & Berger (1999) and
 *     the 4-point kernel of Peskin (2002), both cited in Sec. 3.1;
 *   - markers: N = round(pi (D/h)^2) on an equal-area Fibonacci spiral,
 *     dV = (pi h / 3N)(3 D^2 + h^2) (the shell of thickness h split evenly);
 *   - stencil: s = (X - lo)/h per axis; owning cell floor(s); stencil base
 *     floor(s) - 1 (P = 3) or floor(s - 1/2) - 1 (P = 4); stencil cells are
 *     base + a, a = 0..P-1, wrapped when the axis is periodic; kernel
 *     argument r = s - (base + a) - 1/2;
 *   - Algorithm 1 runs over all markers of all particles together (Jacobi);
 *     F^0 = 0; f^m is recomputed from zero every iteration.  A particle-by-
 *     particle ("sequential") variant is provided for comparison.
 *
 * parity unpinned: the Fibonacci spiral's orientation is fixed by the reading
 * above, not by the paper.  The sequential variant is pinned by composition
 * (two overlapping particles = the first one's loop, then the second one's
 * loop on the field the first left).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IBO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Regularized delta kernels (Sec. 3.1, Algorithm 1: "three-point or        */
/* four-point delta function"; kernels of the cited Roma 1999 / Peskin 2002) */
/* ------------------------------------------------------------------------ */

/* Roma-Peskin-Berger 3-point kernel, support |r| <= 3/2. */
double ibo_phi3(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5) {
        double t = 1.0 - a;
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * t * t)) / 6.0;
    }
    return 0.0;
}

/* Peskin 4-point kernel, support |r| <= 2. */
double ibo_phi4(double r)
{
    double a = fabs(r);
    if (a <= 1.0)
        return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0)
        return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* Derivatives d(phi)/dr of the two kernels (both are C^1). */
double ibo_dphi3(double r)
{
    double a = fabs(r), sg = (r < 0.0) ? -1.0 : 1.0, d;
    if (a <= 0.5)
        d = -a / sqrt(1.0 - 3.0 * a * a);
    else if (a <= 1.5) {
        double t = 1.0 - a;
        d = (-3.0 - 3.0 * t / sqrt(1.0 - 3.0 * t * t)) / 6.0;
    } else
        d = 0.0;
    return sg * d;
}

double ibo_dphi4(double r)
{
    double a = fabs(r), sg = (r < 0.0) ? -1.0 : 1.0, d;
    if (a <= 1.0)
        d = (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    else if (a <= 2.0)
        d = (-2.0 - (6.0 - 4.0 * a) / sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    else
        d = 0.0;
    return sg * d;
}

double ibo_phi(int P, double r) { return P == 3 ? ibo_phi3(r) : ibo_phi4(r); }
double ibo_dphi(int P, double r) { return P == 3 ? ibo_dphi3(r) : ibo_dphi4(r); }

/* ------------------------------------------------------------------------ */
/* Grid description                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n[3];
    double h;
    double lo[3];
    int32_t periodic[3];
} ibo_grid;

static int64_t cells_total(const ibo_grid* g)
{
    return (int64_t)g->n[0] * g->n[1] * g->n[2];
}

static int64_t lin(const ibo_grid* g, int64_t i, int64_t j, int64_t k)
{
    return i + (int64_t)g->n[0] * (j + (int64_t)g->n[1] * k);
}

static int64_t wrap(int64_t i, int32_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

/* Threads of the loops below: sets the count (OpenMP build) and returns it;
 * always 1 in the single-threaded build. */
int ibo_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* z planes [z0, z1) owned by the calling thread inside a parallel region
 * (the whole grid outside one, or in the single-threaded build). */
static void thread_slab(const ibo_grid* g, int64_t* z0, int64_t* z1)
{
#ifdef _OPENMP
    int64_t t = omp_get_thread_num(), nt = omp_get_num_threads();
#else
    int64_t t = 0, nt = 1;
#endif
    *z0 = (int64_t)g->n[2] * t / nt;
    *z1 = (int64_t)g->n[2] * (t + 1) / nt;
}

/* Grid coordinate s = (X - lo)/h of one axis (cell i spans [i, i+1)). */
static double grid_coord(const ibo_grid* g, int axis, double X)
{
    return (X - g->lo[axis]) / g->h;
}

/* Stencil base of one axis (index conventions in the header comment). */
static int64_t stencil_base(int P, double s)
{
    return P == 3 ? (int64_t)floor(s) - 1 : (int64_t)floor(s - 0.5) - 1;
}

/* One axis of the delta stencil: wrapped cell indices and kernel weights.
 * Returns 0, or -1 when a cell leaves a non-periodic axis. */
static int stencil_axis(const ibo_grid* g, int P, int axis, double X,
                        int64_t* cells, double* w, double* r_out)
{
    double s = grid_coord(g, axis, X);
    int64_t b = stencil_base(P, s);
    for (int a = 0; a < P; ++a) {
        int64_t c = b + a;
        double r = s - (double)c - 0.5;
        if (g->periodic[axis])
            c = wrap(c, g->n[axis]);
        else if (c < 0 || c >= g->n[axis])
            return -1;
        cells[a] = c;
        w[a] = ibo_phi(P, r);
        if (r_out)
            r_out[a] = r;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* a1: Lagrangian markers on each sphere surface (Sec. 3.1: markers only on */
/* the particle surface, finest level).                                     */
/* ------------------------------------------------------------------------ */

/* offs[np+1] (host); returns the total marker count. */
int64_t ibo_count_markers(int32_t np, const double* d, double h, int64_t* offs)
{
    offs[0] = 0;
    for (int32_t p = 0; p < np; ++p) {
        double q = d[p] / h;
        offs[p + 1] = offs[p] + (int64_t)llround(IBO_PI * q * q);
    }
    return offs[np];
}

void ibo_build_markers(int32_t np, const double* xc, const double* d, double h,
                       const int64_t* offs, double* x, double* y, double* z,
                       int32_t* pid, double* dv)
{
    double golden = IBO_PI * (3.0 - sqrt(5.0));
    for (int32_t p = 0; p < np; ++p) {
        int64_t N = offs[p + 1] - offs[p];
        double R = 0.5 * d[p];
        dv[p] = IBO_PI * h / (3.0 * (double)N) * (3.0 * d[p] * d[p] + h * h);
        for (int64_t l = 0; l < N; ++l) {
            double zl = 1.0 - (2.0 * (double)l + 1.0) / (double)N;
            double rho = sqrt(1.0 - zl * zl);
            double th = (double)l * golden;
            int64_t m = offs[p] + l;
            x[m] = xc[3 * p + 0] + R * (rho * cos(th));
            y[m] = xc[3 * p + 1] + R * (rho * sin(th));
            z[m] = xc[3 * p + 2] + R * zl;
            pid[m] = p;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* a2: bucketing of markers by owning 8^3 tile (stable counting sort) and   */
/* the per-tile list of markers whose stencil touches the tile.            */
/* Not in the paper, which loops over particles one at a time.             */
/* ------------------------------------------------------------------------ */

/* Returns the number of markers whose stencil leaves the covered boxes or a
 * non-periodic axis (0 = all fine).  lut: box id per box (x fastest), -1 for
 * uncovered, or NULL when every box is covered. */
int64_t ibo_bucket(const int32_t* n, const double* lo, double h, const int32_t* periodic,
                   int32_t box, const int32_t* lut, int32_t tile, int32_t P,
                   int64_t nl, const double* x, const double* y, const double* z,
                   int32_t* cell, int32_t* tileid, int32_t* base, int32_t* perm,
                   int32_t* tile_offs, int32_t* src_offs, int32_t* src_idx,
                   int64_t src_cap, int64_t* nsrc_out)
{
    ibo_grid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.lo[a] = lo[a];
        g.periodic[a] = periodic[a];
    }
    g.h = h;
    int32_t nt[3] = {n[0] / tile, n[1] / tile, n[2] / tile};
    int64_t T = (int64_t)nt[0] * nt[1] * nt[2];
    int32_t nb[3] = {n[0] / box, n[1] / box, n[2] / box};
    int64_t flagged = 0;
    const double* X[3] = {x, y, z};

    /* owning cell, tile, stencil base, coverage flag */
    for (int64_t l = 0; l < nl; ++l) {
        int64_t c[3];
        int bad = 0;
        for (int a = 0; a < 3; ++a) {
            double s = grid_coord(&g, a, X[a][l]);
            int64_t fl = (int64_t)floor(s);
            base[3 * l + a] = (int32_t)stencil_base(P, s);
            c[a] = periodic[a] ? wrap(fl, n[a]) : fl;
            if (c[a] < 0 || c[a] >= n[a]) {
                bad = 1;
                c[a] = c[a] < 0 ? 0 : n[a] - 1;
            }
        }
        cell[l] = (int32_t)lin(&g, c[0], c[1], c[2]);
        tileid[l] = (int32_t)((c[0] / tile) + (int64_t)nt[0] * ((c[1] / tile) + (int64_t)nt[1] * (c[2] / tile)));
        /* every stencil cell must exist and lie in a covered box */
        for (int k = 0; k < P && !bad; ++k)
            for (int j = 0; j < P && !bad; ++j)
                for (int i = 0; i < P && !bad; ++i) {
                    int64_t q[3] = {base[3 * l] + i, base[3 * l + 1] + j, base[3 * l + 2] + k};
                    for (int a = 0; a < 3; ++a) {
                        if (periodic[a])
                            q[a] = wrap(q[a], n[a]);
                        else if (q[a] < 0 || q[a] >= n[a])
                            bad = 1;
                    }
                    if (!bad && lut) {
                        int64_t bi = (q[0] / box) + (int64_t)nb[0] * ((q[1] / box) + (int64_t)nb[1] * (q[2] / box));
                        if (lut[bi] < 0)
                            bad = 1;
                    }
                }
        flagged += bad;
    }

    /* stable counting sort by tile: histogram, exclusive scan, scatter */
    memset(tile_offs, 0, sizeof(int32_t) * (size_t)(T + 1));
    for (int64_t l = 0; l < nl; ++l)
        tile_offs[tileid[l] + 1]++;
    for (int64_t t = 0; t < T; ++t)
        tile_offs[t + 1] += tile_offs[t];
    int32_t* cursor = (int32_t*)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    memcpy(cursor, tile_offs, sizeof(int32_t) * (size_t)T);
    for (int64_t l = 0; l < nl; ++l)
        perm[cursor[tileid[l]]++] = (int32_t)l;

    /* per tile: sorted positions of markers whose stencil touches the tile */
    memset(src_offs, 0, sizeof(int32_t) * (size_t)(T + 1));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t t = 0; t < T; ++t)
                src_offs[t + 1] += src_offs[t];
            memcpy(cursor, src_offs, sizeof(int32_t) * (size_t)T);
        }
        for (int64_t i = 0; i < nl; ++i) {
            int64_t l = perm[i];
            int64_t tl[3][2];
            int ntl[3];
            for (int a = 0; a < 3; ++a) {
                ntl[a] = 0;
                for (int o = 0; o < P; ++o) {
                    int64_t q = base[3 * l + a] + o;
                    if (periodic[a])
                        q = wrap(q, n[a]);
                    if (q < 0 || q >= n[a])
                        continue;
                    int64_t tq = q / tile;
                    int seen = 0;
                    for (int e = 0; e < ntl[a]; ++e)
                        seen |= (tl[a][e] == tq);
                    if (!seen && ntl[a] < 2)
                        tl[a][ntl[a]++] = tq;
                }
            }
            for (int kk = 0; kk < ntl[2]; ++kk)
                for (int jj = 0; jj < ntl[1]; ++jj)
                    for (int ii = 0; ii < ntl[0]; ++ii) {
                        int64_t t = tl[0][ii] + (int64_t)nt[0] * (tl[1][jj] + (int64_t)nt[1] * tl[2][kk]);
                        if (pass == 0)
                            src_offs[t + 1]++;
                        else if (cursor[t] < src_cap)
                            src_idx[cursor[t]++] = (int32_t)i;
                    }
        }
    }
    *nsrc_out = src_offs[T];
    free(cursor);
    return flagged;
}

/* ------------------------------------------------------------------------ */
/* a3: desired marker velocity, Eq. (pr1): U^d = U_r + W_r x (X_l - X_r).   */
/* ------------------------------------------------------------------------ */

void ibo_desired_velocity(int64_t nl, const double* x, const double* y, const double* z,
                          const int32_t* pid, const double* xc, const double* up,
                          const double* om, double* Ud)
{
    for (int64_t l = 0; l < nl; ++l) {
        int p = pid[l];
        double R[3] = {x[l] - xc[3 * p], y[l] - xc[3 * p + 1], z[l] - xc[3 * p + 2]};
        const double* w = om + 3 * p;
        Ud[3 * l + 0] = up[3 * p + 0] + (w[1] * R[2] - w[2] * R[1]);
        Ud[3 * l + 1] = up[3 * p + 1] + (w[2] * R[0] - w[0] * R[2]);
        Ud[3 * l + 2] = up[3 * p + 2] + (w[0] * R[1] - w[1] * R[0]);
    }
}

/* ------------------------------------------------------------------------ */
/* a4: velocity interpolation (Algorithm 1, "Interpolate Lagrangian         */
/* Velocity"): U_l = sum_x u(x) delta_h(x - X_l) h^3, delta_h h^3 = prod phi. */
/* ------------------------------------------------------------------------ */

static int interp_one(const ibo_grid* g, int P, double X, double Y, double Z,
                      const double* u, double U[3])
{
    int64_t ci[3][4];
    double w[3][4];
    const double P3[3] = {X, Y, Z};
    for (int a = 0; a < 3; ++a)
        if (stencil_axis(g, P, a, P3[a], ci[a], w[a], NULL))
            return -1;
    int64_t N = cells_total(g);
    U[0] = U[1] = U[2] = 0.0;
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                double wt = w[0][i] * w[1][j] * w[2][k];
                int64_t q = lin(g, ci[0][i], ci[1][j], ci[2][k]);
                for (int c = 0; c < 3; ++c)
                    U[c] += u[c * N + q] * wt;
            }
    return 0;
}

int ibo_interp(const ibo_grid* g, int P, int64_t nl, const double* x, const double* y,
               const double* z, const double* u, double* U)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t l = 0; l < nl; ++l)
        if (interp_one(g, P, x[l], y[l], z[l], u, U + 3 * l))
            bad = 1;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* a6: force spreading (Algorithm 1, "Spreading Lagrangian Force onto        */
/* Eulerian Force"): f(x) = sum_l F_l delta_h(x - X_l) dV_l.                */
/* f is zeroed first: f^m is built from scratch each iteration.            */
/* ------------------------------------------------------------------------ */

/* Adds marker l's contribution to the cells of f whose z plane lies in
 * [z0, z1) (the calling thread's slab). */
static int spread_add(const ibo_grid* g, int P, double X, double Y, double Z,
                      const double V[3], double scale, double* f, int64_t z0, int64_t z1)
{
    int64_t ci[3][4];
    double w[3][4];
    const double P3[3] = {X, Y, Z};
    for (int a = 0; a < 3; ++a)
        if (stencil_axis(g, P, a, P3[a], ci[a], w[a], NULL))
            return -1;
    int64_t N = cells_total(g);
    for (int k = 0; k < P; ++k) {
        if (ci[2][k] < z0 || ci[2][k] >= z1)
            continue;
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                double wt = w[0][i] * w[1][j] * w[2][k] * scale;
                int64_t q = lin(g, ci[0][i], ci[1][j], ci[2][k]);
                for (int c = 0; c < 3; ++c)
                    f[c * N + q] += V[c] * wt;
            }
    }
    return 0;
}

/* f = sum over markers [l0, l1) of F_l dV_l delta_h, from zero.  Each thread
 * owns a slab of z planes and visits every marker in index order. */
static int spread_range(const ibo_grid* g, int P, int64_t l0, int64_t l1, const double* x,
                        const double* y, const double* z, const int32_t* pid,
                        const double* dv, const double* F, double* f)
{
    int64_t N = cells_total(g);
    double h3 = g->h * g->h * g->h;
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < 3 * N; ++q)
        f[q] = 0.0;
#pragma omp parallel reduction(| : bad)
    {
        int64_t z0, z1;
        thread_slab(g, &z0, &z1);
        for (int64_t l = l0; l < l1; ++l)
            if (spread_add(g, P, x[l], y[l], z[l], F + 3 * l, dv[pid[l]] / h3, f, z0, z1))
                bad = 1;
    }
    return bad ? -1 : 0;
}

int ibo_spread(const ibo_grid* g, int P, int64_t nl, const double* x, const double* y,
               const double* z, const int32_t* pid, const double* dv, const double* F,
               double* f)
{
    return spread_range(g, P, 0, nl, x, y, z, pid, dv, F, f);
}

/* ------------------------------------------------------------------------ */
/* a4-a9: Algorithm 1 (multidirect forcing).                                 */
/*   u^(0) = u0; for m = 1..Ns: U = J u^(m-1); F^m = F^(m-1) + (U^d - U)/dt; */
/*   f^m = S F^m; u^(m) = u0 + dt f^m.  Outputs u* = u^(Ns), f^Ns, F^Ns.     */
/* resid[m] = sqrt(sum_l dV_l |U^d_l - (J u^(m))_l|^2), m = 0..Ns.           */
/* Fhist (optional) receives F^1..F^Ns for the reverse sweep.               */
/* order = 0: all markers together; order = 1: particle by particle, each   */
/* particle starting from the field left by the previous one.              */
/* ------------------------------------------------------------------------ */

static double residual(const ibo_grid* g, int P, int64_t l0, int64_t l1, const double* x,
                       const double* y, const double* z, const int32_t* pid,
                       const double* dv, const double* Ud, const double* u)
{
    /* the errors are formed per marker (in parallel), then summed in index order */
    int64_t n = l1 - l0;
    double* e = (double*)malloc(sizeof(double) * (size_t)(3 * (n > 0 ? n : 1)));
#pragma omp parallel for schedule(static)
    for (int64_t l = l0; l < l1; ++l) {
        double U[3];
        interp_one(g, P, x[l], y[l], z[l], u, U);
        for (int c = 0; c < 3; ++c)
            e[3 * (l - l0) + c] = Ud[3 * l + c] - U[c];
    }
    double acc = 0.0;
    for (int64_t l = l0; l < l1; ++l)
        for (int c = 0; c < 3; ++c) {
            double ec = e[3 * (l - l0) + c];
            acc += dv[pid[l]] * ec * ec;
        }
    free(e);
    return sqrt(acc);
}

/* One multidirect loop over the marker range [l0, l1), starting from field
 * ustart; writes u^(Ns) into ucur and f^Ns into fpart. */
static int multidirect_range(const ibo_grid* g, int P, int ns, double dt, int64_t l0,
                             int64_t l1, const double* x, const double* y, const double* z,
                             const int32_t* pid, const double* dv, const double* Ud,
                             const double* ustart, double* ucur, double* fpart, double* F,
                             double* Fhist, int64_t nl, double* resid)
{
    int64_t N = cells_total(g);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < 3 * N; ++q)
        ucur[q] = ustart[q];
    for (int64_t l = l0; l < l1; ++l)
        F[3 * l] = F[3 * l + 1] = F[3 * l + 2] = 0.0;
    if (resid)
        resid[0] = residual(g, P, l0, l1, x, y, z, pid, dv, Ud, ucur);
    for (int m = 1; m <= ns; ++m) {
        /* interpolate u^(m-1) and update the Lagrangian force */
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t l = l0; l < l1; ++l) {
            double U[3];
            if (interp_one(g, P, x[l], y[l], z[l], ucur, U)) {
                bad = 1;
                continue;
            }
            for (int c = 0; c < 3; ++c)
                F[3 * l + c] = F[3 * l + c] + (Ud[3 * l + c] - U[c]) / dt;
        }
        if (bad)
            return -1;
        if (Fhist)
            for (int64_t l = l0; l < l1; ++l)
                for (int c = 0; c < 3; ++c)
                    Fhist[((int64_t)(m - 1) * nl + l) * 3 + c] = F[3 * l + c];
        /* spread F^m from scratch */
        if (spread_range(g, P, l0, l1, x, y, z, pid, dv, F, fpart))
            return -1;
        /* correct the velocity: u^(m) = u^(0) + dt f^m */
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 3 * N; ++q)
            ucur[q] = ustart[q] + dt * fpart[q];
        if (resid)
            resid[m] = residual(g, P, l0, l1, x, y, z, pid, dv, Ud, ucur);
    }
    return 0;
}

int ibo_multidirect(const ibo_grid* g, int P, int ns, double dt, int order, int32_t np,
                    const int64_t* offs, const double* xc, const double* up, const double* om,
                    int64_t nl, const double* x, const double* y, const double* z,
                    const int32_t* pid, const double* dv, const double* u0, double* ustar,
                    double* f, double* F, double* Fhist, double* resid)
{
    int64_t N = cells_total(g);
    double* Ud = (double*)malloc(sizeof(double) * (size_t)(3 * (nl > 0 ? nl : 1)));
    ibo_desired_velocity(nl, x, y, z, pid, xc, up, om, Ud);
    int rc = 0;
    if (order == 0) {
        rc = multidirect_range(g, P, ns, dt, 0, nl, x, y, z, pid, dv, Ud, u0, ustar, f, F,
                               Fhist, nl, resid);
    } else {
        double* ustart = (double*)malloc(sizeof(double) * (size_t)(3 * N));
        double* fp = (double*)malloc(sizeof(double) * (size_t)(3 * N));
        memcpy(ustar, u0, sizeof(double) * (size_t)(3 * N));
        memset(f, 0, sizeof(double) * (size_t)(3 * N));
        for (int32_t p = 0; p < np && rc == 0; ++p) {
            memcpy(ustart, ustar, sizeof(double) * (size_t)(3 * N));
            rc = multidirect_range(g, P, ns, dt, offs[p], offs[p + 1], x, y, z, pid, dv, Ud,
                                   ustart, ustar, fp, F, Fhist, nl, NULL);
            for (int64_t q = 0; q < 3 * N; ++q)
                f[q] += fp[q];
        }
        free(ustart);
        free(fp);
    }
    free(Ud);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* a10: per-particle sums for the rigid-body update, Eqs. (particle1),      */
/* (particle2) and (FD): sum F dV, sum R x F dV, int u dV, int r x u dV.     */
/* The volume integrals use the particle volume fraction alpha of Eq.       */
/* (level-set function) from the eight nodal level-set values, with the    */
/* scaled level set of the ellipsoid equation (semi-axes equal for a        */
/* sphere).  Raw sums are returned; the caller applies -rho_f.              */
/* ------------------------------------------------------------------------ */

/* alpha of the cell whose low node is (i, j, k) (unwrapped grid indices),
 * for the ellipsoid centred at c with semi-axes ax[3]. */
static double pvf_alpha(const ibo_grid* g, int64_t i, int64_t j, int64_t k,
                        const double* c, const double* ax)
{
    double num = 0.0, den = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                double xn = g->lo[0] + (double)(i + di) * g->h;
                double yn = g->lo[1] + (double)(j + dj) * g->h;
                double zn = g->lo[2] + (double)(k + dk) * g->h;
                double ex = (xn - c[0]) / ax[0], ey = (yn - c[1]) / ax[1], ez = (zn - c[2]) / ax[2];
                double phi = sqrt(ex * ex + ey * ey + ez * ez) - 1.0;
                /* H(-phi) = 1 when -phi > 0, i.e. the node is inside */
                if (-phi > 0.0)
                    num += -phi;
                den += fabs(phi);
            }
    return den > 0.0 ? num / den : 0.0;
}

/* Bounding index range of a body: [floor(s - e) - 1, floor(s + e) + 1]. */
static void body_range(const ibo_grid* g, int axis, double c, double extent, int64_t* i0,
                       int64_t* i1)
{
    double s = grid_coord(g, axis, c);
    double e = extent / g->h;
    *i0 = (int64_t)floor(s - e) - 1;
    *i1 = (int64_t)floor(s + e) + 1;
}

/* Volume sum alpha h^3 of one ellipsoid (Tables 1 and 2 of Sec. 4.1). */
double ibo_pvf_volume(const ibo_grid* g, const double* c, const double* ax)
{
    int64_t r0[3], r1[3];
    for (int a = 0; a < 3; ++a)
        body_range(g, a, c[a], ax[a], &r0[a], &r1[a]);
    double h3 = g->h * g->h * g->h, vol = 0.0;
    for (int64_t k = r0[2]; k <= r1[2]; ++k)
        for (int64_t j = r0[1]; j <= r1[1]; ++j)
            for (int64_t i = r0[0]; i <= r1[0]; ++i)
                vol += pvf_alpha(g, i, j, k, c, ax) * h3;
    return vol;
}

int ibo_particle_reductions(const ibo_grid* g, int32_t np, const double* xc, const double* d,
                            const int64_t* offs, const double* x, const double* y,
                            const double* z, const double* dv, const double* F,
                            const double* u, double* out)
{
    int64_t N = cells_total(g);
    double h3 = g->h * g->h * g->h;
    for (int32_t p = 0; p < np; ++p) {
        double* o = out + 12 * p;
        for (int q = 0; q < 12; ++q)
            o[q] = 0.0;
        const double* c = xc + 3 * p;
        /* Lagrangian sums: sum F dV and sum R x F dV */
        for (int64_t l = offs[p]; l < offs[p + 1]; ++l) {
            const double* Fl = F + 3 * l;
            double R[3] = {x[l] - c[0], y[l] - c[1], z[l] - c[2]};
            for (int a = 0; a < 3; ++a)
                o[a] += Fl[a] * dv[p];
            o[3] += (R[1] * Fl[2] - R[2] * Fl[1]) * dv[p];
            o[4] += (R[2] * Fl[0] - R[0] * Fl[2]) * dv[p];
            o[5] += (R[0] * Fl[1] - R[1] * Fl[0]) * dv[p];
        }
        /* Eulerian volume integrals weighted by alpha */
        double R = 0.5 * d[p], ax[3] = {R, R, R};
        int64_t r0[3], r1[3];
        for (int a = 0; a < 3; ++a)
            body_range(g, a, c[a], R, &r0[a], &r1[a]);
        for (int64_t k = r0[2]; k <= r1[2]; ++k)
            for (int64_t j = r0[1]; j <= r1[1]; ++j)
                for (int64_t i = r0[0]; i <= r1[0]; ++i) {
                    double al = pvf_alpha(g, i, j, k, c, ax);
                    if (al == 0.0)
                        continue;
                    int64_t q[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a) {
                        if (g->periodic[a])
                            q[a] = wrap(q[a], g->n[a]);
                        else if (q[a] < 0 || q[a] >= g->n[a])
                            return -1;
                    }
                    int64_t cq = lin(g, q[0], q[1], q[2]);
                    double uc[3] = {u[cq], u[N + cq], u[2 * N + cq]};
                    double r[3] = {g->lo[0] + ((double)i + 0.5) * g->h - c[0],
                                   g->lo[1] + ((double)j + 0.5) * g->h - c[1],
                                   g->lo[2] + ((double)k + 0.5) * g->h - c[2]};
                    double wgt = al * h3;
                    for (int a = 0; a < 3; ++a)
                        o[6 + a] += uc[a] * wgt;
                    o[9] += (r[1] * uc[2] - r[2] * uc[1]) * wgt;
                    o[10] += (r[2] * uc[0] - r[0] * uc[2]) * wgt;
                    o[11] += (r[0] * uc[1] - r[1] * uc[0]) * wgt;
                }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* a11: reverse sweep of Algorithm 1 (Euclidean vector-Jacobian product).   */
/* S and J are adjoint (Sec. 2), so the transpose of spreading is an        */
/* interpolation weighted by dV/h^3 and the transpose of interpolation is a */
/* spreading without dV.  Gradients with respect to the marker positions    */
/* use d(phi)/dr.  u^(m-1) is recomputed from u0 + dt S F^(m-1).             */
/* ------------------------------------------------------------------------ */

/* Xbar_l += scale * sum_x (fld(x) . v) grad_X w_l(x). */
static int grad_pos(const ibo_grid* g, int P, double X, double Y, double Z,
                    const double* fld, const double v[3], double scale, double out[3])
{
    int64_t ci[3][4];
    double w[3][4], r[3][4], dw[3][4];
    const double P3[3] = {X, Y, Z};
    for (int a = 0; a < 3; ++a) {
        if (stencil_axis(g, P, a, P3[a], ci[a], w[a], r[a]))
            return -1;
        /* r = s - cell centre = (X - x_cell)/h, so d r / d X = 1/h */
        for (int o = 0; o < P; ++o)
            dw[a][o] = ibo_dphi(P, r[a][o]) / g->h;
    }
    int64_t N = cells_total(g);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                int64_t q = lin(g, ci[0][i], ci[1][j], ci[2][k]);
                double dot = fld[q] * v[0] + fld[N + q] * v[1] + fld[2 * N + q] * v[2];
                out[0] += scale * dot * dw[0][i] * w[1][j] * w[2][k];
                out[1] += scale * dot * w[0][i] * dw[1][j] * w[2][k];
                out[2] += scale * dot * w[0][i] * w[1][j] * dw[2][k];
            }
    return 0;
}

int ibo_reverse(const ibo_grid* g, int P, int ns, double dt, int32_t np, const int64_t* offs,
                const double* xc, const double* up, const double* om, int64_t nl,
                const double* x, const double* y, const double* z, const int32_t* pid,
                const double* dv, const double* u0, const double* Fhist, const double* gus,
                const double* gf, const double* gF, double* gu0, double* gup, double* gom,
                double* gX)
{
    int64_t N = cells_total(g);
    double h3 = g->h * g->h * g->h;
    size_t fb = sizeof(double) * (size_t)(3 * N), mb = sizeof(double) * (size_t)(3 * (nl > 0 ? nl : 1));
    double* au = (double*)calloc(3 * N, sizeof(double));     /* adjoint of u^(m) */
    double* af = (double*)calloc(3 * N, sizeof(double));     /* adjoint of f^m */
    double* aF = (double*)calloc(3 * (nl > 0 ? nl : 1), sizeof(double)); /* adjoint of F^m */
    double* aUd = (double*)calloc(3 * (nl > 0 ? nl : 1), sizeof(double));
    double* Ub = (double*)malloc(mb);
    double* uprev = (double*)malloc(fb);
    double* fprev = (double*)malloc(fb);
    int rc = 0;
    memset(gu0, 0, fb);
    memset(gX, 0, mb);
    if (gus)
        memcpy(au, gus, fb);
    if (gf)
        memcpy(af, gf, fb);
    if (gF)
        memcpy(aF, gF, mb);
    for (int m = ns; m >= 1 && rc == 0; --m) {
        const double* Fm = Fhist + (int64_t)(m - 1) * nl * 3;
        /* u^(m) = u0 + dt f^m */
        for (int64_t q = 0; q < 3 * N; ++q) {
            gu0[q] += au[q];
            af[q] += dt * au[q];
        }
        /* f^m = S[X] F^m */
        for (int64_t l = 0; l < nl && rc == 0; ++l) {
            double s = dv[pid[l]] / h3, Ut[3];
            rc |= interp_one(g, P, x[l], y[l], z[l], af, Ut);
            for (int c = 0; c < 3; ++c)
                aF[3 * l + c] += s * Ut[c];
            rc |= grad_pos(g, P, x[l], y[l], z[l], af, Fm + 3 * l, s, gX + 3 * l);
        }
        /* F^m = F^(m-1) + (U^d - U^m)/dt */
        for (int64_t q = 0; q < 3 * nl; ++q) {
            aUd[q] += aF[q] / dt;
            Ub[q] = -aF[q] / dt;
        }
        /* U^m = J[X] u^(m-1), with u^(m-1) = u0 + dt S F^(m-1) recomputed */
        if (m == 1)
            memcpy(uprev, u0, fb);
        else {
            rc |= ibo_spread(g, P, nl, x, y, z, pid, dv, Fhist + (int64_t)(m - 2) * nl * 3, fprev);
            for (int64_t q = 0; q < 3 * N; ++q)
                uprev[q] = u0[q] + dt * fprev[q];
        }
        memset(au, 0, fb);
        for (int64_t l = 0; l < nl && rc == 0; ++l) {
            rc |= spread_add(g, P, x[l], y[l], z[l], Ub + 3 * l, 1.0, au, 0, g->n[2]);
            rc |= grad_pos(g, P, x[l], y[l], z[l], uprev, Ub + 3 * l, 1.0, gX + 3 * l);
        }
        memset(af, 0, fb);
    }
    for (int64_t q = 0; q < 3 * N; ++q)
        gu0[q] += au[q];
    /* U^d = U_p + omega x R */
    for (int32_t p = 0; p < np; ++p)
        for (int c = 0; c < 3; ++c)
            gup[3 * p + c] = gom[3 * p + c] = 0.0;
    for (int64_t l = 0; l < nl; ++l) {
        int p = pid[l];
        const double* a = aUd + 3 * l;
        const double* w = om + 3 * p;
        double R[3] = {x[l] - xc[3 * p], y[l] - xc[3 * p + 1], z[l] - xc[3 * p + 2]};
        for (int c = 0; c < 3; ++c)
            gup[3 * p + c] += a[c];
        gom[3 * p + 0] += R[1] * a[2] - R[2] * a[1];
        gom[3 * p + 1] += R[2] * a[0] - R[0] * a[2];
        gom[3 * p + 2] += R[0] * a[1] - R[1] * a[0];
        gX[3 * l + 0] += a[1] * w[2] - a[2] * w[1];
        gX[3 * l + 1] += a[2] * w[0] - a[0] * w[2];
        gX[3 * l + 2] += a[0] * w[1] - a[1] * w[0];
    }
    (void)offs;
    (void)up;
    free(au);
    free(af);
    free(aF);
    free(aUd);
    free(Ub);
    free(uprev);
    free(fprev);
    return rc ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* The particle side of a time step (Sec. 3.2; Step 4 of Sec. 3.1).         */
/* ------------------------------------------------------------------------ */

/* Rigid-body update of np spheres.  Free motion follows Eqs. (particle1)   */
/* and (particle2) with their right-hand sides taken at the half step (the  */
/* midpoint rule): the marker force is F^{n+1/2} of Algorithm 1 and the      */
/* time derivatives of the volume integrals are their change over dt:        */
/*   rho_p V_p (U^{n+1} - U^n)/dt = -rho_f S_F + rho_f (I_u' - I_u)/dt        */
/*                                  + (rho_p - rho_f) V_p g + F_c             */
/*   I_p (W^{n+1} - W^n)/dt = -rho_f S_T + rho_f (I_ru' - I_ru)/dt + T_c       */
/* with V_p = pi D^3/6 and I_p = rho_p V_p D^2/10 (solid sphere).  sums_n and */
/* sums_np1 are the per-particle sums [S_F, S_T, I_u, I_ru] at t^n and with  */
/* u^{n+1}; only the volume integrals of sums_np1 are used.  Prescribed      */
/* particles keep U and W.  The centroid then moves by Eq. (pr2):            */
/*   X^{n+1} = X^n + dt/2 (U^n + U^{n+1}).                                   */
void ibo_rigid_update(int32_t np, const double* xc, const double* d, const double* up,
                      const double* om, const double* rho_p, const double* sums_n,
                      const double* sums_np1, const double* Fc, const double* Tc,
                      const int32_t* prescribed, double rho_f, const double* grav, double dt,
                      double* up_new, double* om_new, double* xc_new)
{
    for (int32_t p = 0; p < np; ++p) {
        const double D = d[p];
        const double Vp = IBO_PI * D * D * D / 6.0;
        const double mass = rho_p[p] * Vp;
        const double Ip = mass * D * D / 10.0;
        const double* s0 = sums_n + 12 * p;
        const double* s1 = sums_np1 + 12 * p;
        for (int c = 0; c < 3; ++c) {
            double un = up[3 * p + c], wn = om[3 * p + c];
            double u1 = un, w1 = wn;
            if (!(prescribed && prescribed[p])) {
                double force = -rho_f * s0[c] + rho_f * (s1[6 + c] - s0[6 + c]) / dt +
                               (rho_p[p] - rho_f) * Vp * grav[c] + (Fc ? Fc[3 * p + c] : 0.0);
                double torque = -rho_f * s0[3 + c] + rho_f * (s1[9 + c] - s0[9 + c]) / dt +
                                (Tc ? Tc[3 * p + c] : 0.0);
                u1 = un + dt * force / mass;
                w1 = wn + dt * torque / Ip;
            }
            up_new[3 * p + c] = u1;
            om_new[3 * p + c] = w1;
            xc_new[3 * p + c] = xc[3 * p + c] + 0.5 * dt * (un + u1);
        }
    }
}

/* Markers follow their particle's rigid motion (Eq. (x) with U = U_r +      */
/* W x R): X^{n+1} = X_r^{n+1} + Q R^n, R^n = X^n - X_r^n, Q the rotation by  */
/* the angle |W| dt about W/|W| with W = (W^n + W^{n+1})/2 (Rodrigues'        */
/* formula); Q = identity when W = 0.                                         */
void ibo_advect_markers(int64_t nl, const double* x, const double* y, const double* z,
                        const int32_t* pid, const double* xc_n, const double* xc_np1,
                        const double* om_n, const double* om_np1, double dt, double* xn,
                        double* yn, double* zn)
{
    for (int64_t l = 0; l < nl; ++l) {
        const int p = pid[l];
        double R[3] = {x[l] - xc_n[3 * p], y[l] - xc_n[3 * p + 1], z[l] - xc_n[3 * p + 2]};
        double w[3];
        for (int c = 0; c < 3; ++c)
            w[c] = 0.5 * (om_n[3 * p + c] + om_np1[3 * p + c]);
        double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        double out[3] = {R[0], R[1], R[2]};
        if (wn > 0.0) {
            double k[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
            double th = wn * dt, ct = cos(th), st = sin(th);
            double kxr[3] = {k[1] * R[2] - k[2] * R[1], k[2] * R[0] - k[0] * R[2],
                             k[0] * R[1] - k[1] * R[0]};
            double kdr = k[0] * R[0] + k[1] * R[1] + k[2] * R[2];
            for (int c = 0; c < 3; ++c)
                out[c] = R[c] * ct + kxr[c] * st + k[c] * kdr * (1.0 - ct);
        }
        xn[l] = xc_np1[3 * p] + out[0];
        yn[l] = xc_np1[3 * p + 1] + out[1];
        zn[l] = xc_np1[3 * p + 2] + out[2];
    }
}

/* Repulsive collision force of Eq. (DKT_model), after Breugem (2012):       */
/*   F_c,ij = -(m |g| / eps_c) ((|delta| - D_c)/d_c)^2 delta/|delta|           */
/* for |delta| < D_c and 0 otherwise, delta = X_j - X_i (minimum image on    */
/* periodic axes of length L[a] > 0), D_c = R_i + R_j + h, d_c = h (finest   */
/* spacing).  The paper's case has equal particles; m is taken here as the   */
/* mean of the two masses (rho V, V = pi D^3/6), which keeps F_ij = -F_ji.    */
/* Fc[i] = sum over j != i in ascending j.  The force is central: no torque. */
void ibo_collision_forces(int32_t np, const double* xc, const double* d, const double* rho_p,
                          double gnorm, double h, double eps_c, const double* L, double* Fc)
{
    for (int32_t i = 0; i < np; ++i) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int32_t j = 0; j < np; ++j) {
            if (j == i)
                continue;
            double del[3];
            for (int c = 0; c < 3; ++c) {
                del[c] = xc[3 * j + c] - xc[3 * i + c];
                if (L[c] > 0.0)
                    del[c] -= L[c] * floor(del[c] / L[c] + 0.5);
            }
            double dist = sqrt(del[0] * del[0] + del[1] * del[1] + del[2] * del[2]);
            double Dc = 0.5 * (d[i] + d[j]) + h;
            if (!(dist < Dc) || dist == 0.0)
                continue;
            double mi = rho_p[i] * IBO_PI * d[i] * d[i] * d[i] / 6.0;
            double mj = rho_p[j] * IBO_PI * d[j] * d[j] * d[j] / 6.0;
            double m = 0.5 * (mi + mj);
            double q = (dist - Dc) / h;
            double mag = m * gnorm / eps_c * q * q;
            for (int c = 0; c < 3; ++c)
                f[c] -= mag * del[c] / dist;
        }
        for (int c = 0; c < 3; ++c)
            Fc[3 * i + c] = f[c];
    }
}
