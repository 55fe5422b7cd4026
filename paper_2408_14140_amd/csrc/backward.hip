// backward.hip -- a11: adjoint of Algorithm 1 (reverse sweep).
//
// Forward, per iteration m = 1..ns:  U^m = J[X] u^(m-1);  F^m = F^(m-1) +
// (U^d - U^m)/dt;  f^m = S[X] F^m;  u^(m) = u0 + dt f^m.  With the adjoint
// variables a_u (of u^(m)), a_f (of f^m) and a_F (of F^m), the sweep runs
// m = ns..1:
//   g_u0 += a_u;  a_f += dt a_u
//   a_F  += S^T a_f = (dV/h^3) J a_f;   g_X += (dV/h^3) sum_x (a_f . F^m) grad w
//   a_Ud += a_F/dt;  Ubar = -a_F/dt     (a_F carries over to F^(m-1))
//   u^(m-1) recomputed as u0 + dt S F^(m-1) (u0 for m = 1)
//   g_X  += sum_x (u^(m-1) . Ubar) grad w;   a_u = J^T Ubar;   a_f = 0
// then g_u0 += a_u and, from U^d = U_r + W_r x R (Eq. (pr1)),
//   g_up = sum a_Ud,  g_om = sum R x a_Ud,  g_X += a_Ud x W_r.
// S and J are adjoint (Sec. 2): J^T is spreading without dV and S^T is
// interpolation weighted by dV/h^3.  grad w uses the kernel derivative.
// Fields are recomputed, never stored.  The two spreads of every step (the
// recomputed u^(m-1) and J^T Ubar) run on the forward loop's tile kernel,
// with its marker records and work lists formed once per call (grids of at
// least 16 cells per axis; the plain per-cell kernel otherwise), and so do
// J a_f and the position gradients (the tile interpolation in its adjoint
// mode, J a_f and its gradient in one pass over a_f; four lanes per marker
// gathering from global memory otherwise).
#include "paths.h"

namespace ibx {

// mode 0: a = 0; 1: a = b; 2: a += b; 3: a = u0 + dt b; 4: (a += b, c += dt b);
// 5: (a += b, c = dt b)
template <typename T, int MODE>
__global__ void k_field_op(Grid g, T* __restrict__ a, const T* __restrict__ b,
                           T* __restrict__ c, const T* __restrict__ u0, double dt)
{
    const int64_t per_box = (int64_t)g.box * g.box * g.box;
    const int64_t total = per_box * g.nbox;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bid = q / per_box;
        const int64_t r = q - bid * per_box;
        const int lx = (int)(r % g.box) + g.ngrow;
        const int ly = (int)((r / g.box) % g.box) + g.ngrow;
        const int lz = (int)(r / ((int64_t)g.box * g.box)) + g.ngrow;
        const int64_t off = bid * g.bstride + ((int64_t)lz * g.ext + ly) * g.ext + lx;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t o = off + k * g.cstride;
            if (MODE == 0) a[o] = T(0);
            if (MODE == 1) a[o] = b[o];
            if (MODE == 2) a[o] += b[o];
            if (MODE == 3) a[o] = u0[o] + (T)dt * b[o];
            if (MODE == 4) {
                a[o] += b[o];
                c[o] += (T)dt * b[o];
            }
            if (MODE == 5) {
                a[o] += b[o];
                c[o] = (T)dt * b[o];
            }
        }
    }
}

// Interpolation and position gradient of one field in one pass, four lanes
// per marker (lane k of the four takes the stencil's z planes k, k+4, ...,
// then a fixed shuffle tree sums the four): U_l = J fld (when U is given) and
// gX_l += scale_l * sum over the stencil of (fld(x) . v_l) grad_X w_l(x)
// (when v is given), scale_l = dV_l/h^3 when use_dv, else 1.  A stencil cell
// off a bounded axis or in an uncovered box is skipped (the bucket flags
// report such markers and the call's outputs are poisoned).
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_interp_grad(Grid g, int64_t nl, const double* __restrict__ x, const double* __restrict__ y,
              const double* __restrict__ z, const int32_t* __restrict__ pid,
              const double* __restrict__ dv, const T* __restrict__ fld, T* __restrict__ U,
              const T* __restrict__ v, int use_dv, double* __restrict__ gX)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t l = q >> 2;
    const int sub = (int)(q & 3);
    const bool live = l < nl;
    const int64_t lc = live ? l : 0;
    const double X[3] = {x[lc], y[lc], z[lc]};
    T w[3][P], dw[3][P];
    int c[3][P];
    const T ih = (T)(1.0 / g.h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b = axis_weights_d<T, P>(grid_coord(g, a, X[a]), w[a], dw[a]);
#pragma unroll
        for (int o = 0; o < P; ++o) {
            dw[a][o] *= ih;
            int cq = b + o;
            if (g.periodic[a])
                cq = wrapi(cq, g.n[a]);
            else if (cq < 0 || cq >= g.n[a])
                cq = -1;
            c[a][o] = cq;
        }
    }
    T v0 = T(0), v1 = T(0), v2 = T(0);
    if (v && live) {
        v0 = v[3 * l];
        v1 = v[3 * l + 1];
        v2 = v[3 * l + 2];
    }
    T u0 = 0, u1 = 0, u2 = 0, a0 = 0, a1 = 0, a2 = 0;
    for (int k = sub; live && k < P; k += 4) {
        if (c[2][k] < 0)
            continue;
        for (int j = 0; j < P; ++j) {
            if (c[1][j] < 0)
                continue;
            for (int i = 0; i < P; ++i) {
                if (c[0][i] < 0)
                    continue;
                const int64_t off = cell_offset(g, c[0][i], c[1][j], c[2][k]);
                if (off < 0)
                    continue;
                const T f0 = fld[off], f1 = fld[off + g.cstride], f2 = fld[off + 2 * g.cstride];
                const T wyz = w[1][j] * w[2][k];
                const T wt = w[0][i] * wyz;
                u0 += f0 * wt;
                u1 += f1 * wt;
                u2 += f2 * wt;
                const T dot = f0 * v0 + f1 * v1 + f2 * v2;
                a0 += dot * dw[0][i] * wyz;
                a1 += dot * w[0][i] * dw[1][j] * w[2][k];
                a2 += dot * w[0][i] * w[1][j] * dw[2][k];
            }
        }
    }
    // fixed tree over the four lanes of the marker
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) {
        u0 += __shfl_xor(u0, o);
        u1 += __shfl_xor(u1, o);
        u2 += __shfl_xor(u2, o);
        a0 += __shfl_xor(a0, o);
        a1 += __shfl_xor(a1, o);
        a2 += __shfl_xor(a2, o);
    }
    if (!live || sub != 0)
        return;
    if (U) {
        U[3 * l + 0] = u0;
        U[3 * l + 1] = u1;
        U[3 * l + 2] = u2;
    }
    if (v) {
        const double sc = use_dv ? dv[pid[l]] * g.inv_h3 : 1.0;
        gX[3 * l + 0] += sc * (double)a0;
        gX[3 * l + 1] += sc * (double)a1;
        gX[3 * l + 2] += sc * (double)a2;
    }
}

template <typename T>
static void launch_interp_grad(const Grid& g, int P, const ib_markers* m, const T* fld, T* U,
                               const T* v, int use_dv, double* gX, hipStream_t st)
{
    const int64_t nth = 4 * m->nl;
    const unsigned gb = (unsigned)((nth + 255) / 256);
    if (P == 3)
        k_interp_grad<T, 3><<<gb, 256, 0, st>>>(g, m->nl, m->x, m->y, m->z, m->pid, m->dv, fld,
                                                 U, v, use_dv, gX);
    else
        k_interp_grad<T, 4><<<gb, 256, 0, st>>>(g, m->nl, m->x, m->y, m->z, m->pid, m->dv, fld,
                                                 U, v, use_dv, gX);
}

// a_F += (dV/h^3) Ui;  a_Ud += a_F/dt;  Ubar = -a_F/dt.
template <typename T>
__global__ void k_marker_step(Grid g, int64_t nl, double dt, const int32_t* __restrict__ pid,
                              const double* __restrict__ dv, const T* __restrict__ Ui,
                              T* __restrict__ aF, double* __restrict__ aUd, T* __restrict__ Ub)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    const T sc = (T)(dv[pid[l]] * g.inv_h3);
    const T idt = (T)(1.0 / dt);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T a = aF[3 * l + c] + sc * Ui[3 * l + c];
        aF[3 * l + c] = a;
        aUd[3 * l + c] += (double)a * (1.0 / dt);
        Ub[3 * l + c] = -a * idt;
    }
}

// One workgroup per particle: g_up = sum a_Ud, g_om = sum R x a_Ud (fixed
// tree), and g_X += a_Ud x W_r per marker.
__global__ void __launch_bounds__(256)
k_particle_grads(int32_t np, const int64_t* __restrict__ offs, const double* __restrict__ x,
                 const double* __restrict__ y, const double* __restrict__ z,
                 const double* __restrict__ xc, const double* __restrict__ om,
                 const double* __restrict__ aUd, double* __restrict__ gup,
                 double* __restrict__ gom, double* __restrict__ gX)
{
    __shared__ double red[6][256];
    const int p = blockIdx.x, t = threadIdx.x;
    const double w0 = om[3 * p], w1 = om[3 * p + 1], w2 = om[3 * p + 2];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t l = offs[p] + t; l < offs[p + 1]; l += 256) {
        const double a0 = aUd[3 * l], a1 = aUd[3 * l + 1], a2 = aUd[3 * l + 2];
        const double R0 = x[l] - xc[3 * p], R1 = y[l] - xc[3 * p + 1], R2 = z[l] - xc[3 * p + 2];
        acc[0] += a0;
        acc[1] += a1;
        acc[2] += a2;
        acc[3] += R1 * a2 - R2 * a1;
        acc[4] += R2 * a0 - R0 * a2;
        acc[5] += R0 * a1 - R1 * a0;
        gX[3 * l + 0] += a1 * w2 - a2 * w1;
        gX[3 * l + 1] += a2 * w0 - a0 * w2;
        gX[3 * l + 2] += a0 * w1 - a1 * w0;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
        red[q][t] = acc[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 6; ++q)
                red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t < 3) {
        gup[3 * p + t] = red[t][0];
        gom[3 * p + t] = red[3 + t][0];
    }
}

__global__ void k_zero_d(int64_t n, double* a)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = 0.0;
}

template <typename T>
__global__ void k_copy_or_zero(int64_t n, const T* __restrict__ src, T* __restrict__ dst)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src ? src[q] : T(0);
}

static unsigned grid_n(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

size_t backward_workspace(const Grid& g, ib_prec prec, int64_t nl)
{
    const size_t s = prec == IB_F64 ? 8 : 4;
    Carver cv(nullptr, 0);
    for (int k = 0; k < 3; ++k)
        cv.take<char>(s * field_elems(g));
    for (int k = 0; k < 3; ++k)
        cv.take<char>(s * 3 * nl);
    cv.take<double>(3 * nl);
    if (tile_spread_supported(g))
        cv.take<char>(tile_spread_workspace(g, prec, nl));
    return cv.used;
}

template <typename T>
static int run_backward(const Grid& g, int P, const BatchedCfg& cfg, const ib_particles* p,
                        const ib_markers* m,
                        const ib_buckets* b, int ns, double dt, const T* u0, const T* Fhist,
                        const T* gus, const T* gf, const T* gF, T* gu0, double* gup,
                        double* gom, double* gX, void* ws, size_t ws_bytes, hipStream_t st)
{
    const int64_t nl = m->nl;
    const ib_prec prec = sizeof(T) == 8 ? IB_F64 : IB_F32;
    Carver cv(ws, ws_bytes);
    T* au = cv.take<T>(field_elems(g));
    T* af = cv.take<T>(field_elems(g));
    T* tmp = cv.take<T>(field_elems(g));
    T* aF = cv.take<T>(3 * nl);
    T* Ub = cv.take<T>(3 * nl);
    T* Ui = cv.take<T>(3 * nl);
    double* aUd = cv.take<double>(3 * nl);
    const bool tiled = tile_spread_supported(g);
    const size_t tsb = tiled ? tile_spread_workspace(g, prec, nl) : 0;
    void* tws = tiled ? cv.take<char>(tsb) : nullptr;
    if (!ws || !cv.ok())
        return IB_EWORKSPACE;
    if (tiled) {
        const int rc = tile_spread_setup(g, P, prec, cfg, p, m, b, tws, tsb, st);
        if (rc)
            return rc;
    }
    const unsigned gc = grid_n((int64_t)g.nbox * g.box * g.box * g.box);
    const unsigned gm = grid_n(nl);
    k_field_op<T, 0><<<gc, 256, 0, st>>>(g, gu0, nullptr, nullptr, nullptr, dt);
    if (gus)
        k_field_op<T, 1><<<gc, 256, 0, st>>>(g, au, gus, nullptr, nullptr, dt);
    else
        k_field_op<T, 0><<<gc, 256, 0, st>>>(g, au, nullptr, nullptr, nullptr, dt);
    if (gf)
        k_field_op<T, 1><<<gc, 256, 0, st>>>(g, af, gf, nullptr, nullptr, dt);
    else
        k_field_op<T, 0><<<gc, 256, 0, st>>>(g, af, nullptr, nullptr, nullptr, dt);
    if (nl > 0) {
        k_copy_or_zero<T><<<gm, 256, 0, st>>>(3 * nl, gF, aF);
        k_zero_d<<<gm, 256, 0, st>>>(3 * nl, aUd);
        k_zero_d<<<gm, 256, 0, st>>>(3 * nl, gX);
    }
    for (int mi = ns; mi >= 1; --mi) {
        const T* Fm = Fhist + (int64_t)(mi - 1) * 3 * nl;
        // a_f holds g_f on the first step and nothing afterwards
        if (mi == ns)
            k_field_op<T, 4><<<gc, 256, 0, st>>>(g, gu0, au, af, nullptr, dt);
        else
            k_field_op<T, 5><<<gc, 256, 0, st>>>(g, gu0, au, af, nullptr, dt);
        if (nl > 0) {
            // U = J a_f and the position gradient of S^T with F^m, one gather
            if (tiled) {
                const int rc = tile_interp_grad(g, P, prec, cfg, m, b, af, Fm, Ui, 1, gX, tws,
                                                tsb, st);
                if (rc)
                    return rc;
            } else {
                launch_interp_grad<T>(g, P, m, af, Ui, Fm, 1, gX, st);
            }
            k_marker_step<T><<<gm, 256, 0, st>>>(g, nl, dt, m->pid, m->dv, Ui, aF, aUd, Ub);
        }
        const T* uprev = u0;
        if (mi > 1) {
            const T* Fp = Fhist + (int64_t)(mi - 2) * 3 * nl;
            if (tiled) {
                const int rc = tile_spread(g, P, prec, cfg, m, b, Fp, 1, u0, dt, tmp, tws, tsb, st);
                if (rc)
                    return rc;
            } else {
                plain_spread(g, P, prec, m, b, Fp, tmp, 1.0, 1, st);
                k_field_op<T, 3><<<gc, 256, 0, st>>>(g, tmp, tmp, nullptr, u0, dt);
            }
            uprev = tmp;
        }
        if (nl > 0 && tiled) {
            const int rc = tile_interp_grad(g, P, prec, cfg, m, b, uprev, Ub, nullptr, 0, gX, tws,
                                            tsb, st);
            if (rc)
                return rc;
        } else if (nl > 0) {
            launch_interp_grad<T>(g, P, m, uprev, nullptr, Ub, 0, gX, st);
        }
        if (tiled) {
            const int rc = tile_spread(g, P, prec, cfg, m, b, Ub, 0, nullptr, dt, au, tws, tsb, st);
            if (rc)
                return rc;
        } else {
            plain_spread(g, P, prec, m, b, Ub, au, 1.0, 0, st);
        }
    }
    k_field_op<T, 2><<<gc, 256, 0, st>>>(g, gu0, au, nullptr, nullptr, dt);
    if (p->np > 0)
        k_particle_grads<<<(unsigned)p->np, 256, 0, st>>>(p->np, m->offs, m->x, m->y, m->z,
                                                          p->xc, p->om, aUd, gup, gom, gX);
    return launch_status();
}

int multidirect_backward(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                         const ib_particles* p,
                         const ib_markers* m, const ib_buckets* b, int ns, double dt,
                         const void* u0, const void* Fhist, const void* gus, const void* gf,
                         const void* gF, void* gu0, double* gup, double* gom, double* gX,
                         void* ws, size_t ws_bytes, hipStream_t st)
{
    int rc;
    if (prec == IB_F64)
        rc = run_backward<double>(g, P, cfg, p, m, b, ns, dt, (const double*)u0,
                                  (const double*)Fhist, (const double*)gus, (const double*)gf,
                                  (const double*)gF, (double*)gu0, gup, gom, gX, ws, ws_bytes,
                                  st);
    else
        rc = run_backward<float>(g, P, cfg, p, m, b, ns, dt, (const float*)u0, (const float*)Fhist,
                                 (const float*)gus, (const float*)gf, (const float*)gF,
                                 (float*)gu0, gup, gom, gX, ws, ws_bytes, st);
    if (rc)
        return rc;
    PoisonSet ps;
    ps.field[0] = gu0;
    ps.dvec[0] = gup;
    ps.ndvec[0] = 3 * (int64_t)p->np;
    ps.dvec[1] = gom;
    ps.ndvec[1] = 3 * (int64_t)p->np;
    ps.dvec[2] = gX;
    ps.ndvec[2] = 3 * m->nl;
    poison_if_flagged(b->flag, g, prec, ps, st);
    return launch_status();
}

}  // namespace ibx
