// plain.hip -- the plain path: one kernel per sub-step of Algorithm 1, each
// reading and writing global memory directly (no LDS staging, no fusion).
//   interp   one thread per marker gathers its P^3 stencil
//   force    one thread per marker: F += (U^d - U)/dt
//   spread   one workgroup per 8^3 tile, one thread per cell, pulling the
//            tile's source list in order (deterministic, no atomics)
//   correct  one thread per covered cell: u^(m) = u0 + dt f^m
#include "ibx_internal.h"
#include "paths.h"

namespace ibx {

// Wrapped index on axis a, or -1 outside a bounded axis.
__device__ inline int resolve(const Grid& g, int a, int q)
{
    if (g.periodic[a])
        return wrapi(q, g.n[a]);
    return (q < 0 || q >= g.n[a]) ? -1 : q;
}

template <typename T, int P>
__global__ void __launch_bounds__(256)
k_interp_plain(Grid g, int64_t nl, const double* __restrict__ x, const double* __restrict__ y,
               const double* __restrict__ z, const T* __restrict__ u, T* __restrict__ U)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    const double X[3] = {x[l], y[l], z[l]};
    T w[3][P];
    int c[3][P];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b = axis_weights<T, P>(grid_coord(g, a, X[a]), w[a]);
#pragma unroll
        for (int o = 0; o < P; ++o)
            c[a][o] = resolve(g, a, b + o);
    }
    T acc0 = 0, acc1 = 0, acc2 = 0;
    bool outside = false;     // a stencil cell off a bounded axis or in an uncovered box
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                if ((c[0][i] | c[1][j] | c[2][k]) < 0) {
                    outside = true;
                    continue;
                }
                const int64_t off = cell_offset(g, c[0][i], c[1][j], c[2][k]);
                if (off < 0) {
                    outside = true;
                    continue;
                }
                const T wt = w[0][i] * w[1][j] * w[2][k];
                acc0 += u[off] * wt;
                acc1 += u[off + g.cstride] * wt;
                acc2 += u[off + 2 * g.cstride] * wt;
            }
    if (outside)
        acc0 = acc1 = acc2 = (T)__builtin_nan("");
    U[3 * l + 0] = acc0;
    U[3 * l + 1] = acc1;
    U[3 * l + 2] = acc2;
}

template <typename T>
__global__ void k_force_update(int64_t nl, double dt, const T* __restrict__ Ud,
                               const T* __restrict__ U, T* __restrict__ F,
                               const int32_t* __restrict__ pid, const double* __restrict__ dv,
                               double* e2)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T e = Ud[3 * l + c] - U[3 * l + c];
        F[3 * l + c] = F[3 * l + c] + e / (T)dt;
        acc += (double)e * (double)e;
    }
    if (e2)
        e2[l] = dv[pid[l]] * acc;
}

// e2[l] = dV_l |U^d_l - U_l|^2 without touching F (final residual).
template <typename T>
__global__ void k_resid_only(int64_t nl, const T* __restrict__ Ud, const T* __restrict__ U,
                             const int32_t* __restrict__ pid, const double* __restrict__ dv,
                             double* e2)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double e = (double)Ud[3 * l + c] - (double)U[3 * l + c];
        acc += e * e;
    }
    e2[l] = dv[pid[l]] * acc;
}

// f on one tile: thread = cell; sources visited in list order.
template <typename T, int P>
__global__ void __launch_bounds__(TILE_CELLS)
k_spread_plain(Grid g, const double* __restrict__ x, const double* __restrict__ y,
               const double* __restrict__ z, const int32_t* __restrict__ pid,
               const double* __restrict__ dv, const int32_t* __restrict__ perm,
               const int32_t* __restrict__ src_offs, const int32_t* __restrict__ src_idx,
               const T* __restrict__ F, T* __restrict__ f, T scale, int use_dv)
{
    const int64_t t = blockIdx.x;
    const int tx = (int)(t % g.nt[0]);
    const int ty = (int)((t / g.nt[0]) % g.nt[1]);
    const int tz = (int)(t / ((int64_t)g.nt[0] * g.nt[1]));
    const int cc[3] = {tx * TILE + (int)(threadIdx.x & 7), ty * TILE + (int)((threadIdx.x >> 3) & 7),
                       tz * TILE + (int)(threadIdx.x >> 6)};
    const int64_t off = cell_offset(g, cc[0], cc[1], cc[2]);
    if (off < 0)
        return;  // whole tile lies in an uncovered box
    const double inv_h3 = g.inv_h3;
    T acc0 = 0, acc1 = 0, acc2 = 0;
    const int s0 = src_offs[t], s1 = src_offs[t + 1];
    for (int s = s0; s < s1; ++s) {
        const int64_t l = perm[src_idx[s]];
        const double X[3] = {x[l], y[l], z[l]};
        T wt = T(1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double sa = grid_coord(g, a, X[a]);
            const int b = stencil_base<P>(sa);
            const int d = g.periodic[a] ? wrapi(cc[a] - b, g.n[a]) : cc[a] - b;
            if (d < 0 || d >= P) {
                wt = T(0);
                break;
            }
            wt *= kphi<T, P>((T)(sa - (double)(b + d) - 0.5));
        }
        if (wt != T(0)) {
            wt *= (use_dv ? (T)(dv[pid[l]] * inv_h3) : T(1)) * scale;
            acc0 += F[3 * l + 0] * wt;
            acc1 += F[3 * l + 1] * wt;
            acc2 += F[3 * l + 2] * wt;
        }
    }
    f[off] = acc0;
    f[off + g.cstride] = acc1;
    f[off + 2 * g.cstride] = acc2;
}

// Every valid cell of every covered box: u = u0 + dt f (f may be null: u = u0).
template <typename T>
__global__ void k_correct(Grid g, double dt, const T* __restrict__ u0, const T* __restrict__ f,
                          T* __restrict__ u)
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
        for (int c = 0; c < 3; ++c) {
            const int64_t o = off + c * g.cstride;
            u[o] = f ? u0[o] + (T)dt * f[o] : u0[o];
        }
    }
}

template <typename T>
__global__ void k_zero_field(Grid g, T* __restrict__ f)
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
        f[off] = T(0);
        f[off + g.cstride] = T(0);
        f[off + 2 * g.cstride] = T(0);
    }
}

template <typename T>
__global__ void k_zero_vec(int64_t n, T* __restrict__ a)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = T(0);
}

template <typename T>
__global__ void k_copy_vec(int64_t n, const T* __restrict__ a, T* __restrict__ b)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        b[q] = a[q];
}

// Deterministic sum of squares: fixed chunking, fixed tree.
constexpr int RED_THREADS = 256;
constexpr int RED_CHUNK = RED_THREADS * 16;

__global__ void __launch_bounds__(RED_THREADS)
k_sum_partial(const double* __restrict__ v, int64_t n, double* __restrict__ part)
{
    __shared__ double s[RED_THREADS];
    const int64_t base = (int64_t)blockIdx.x * RED_CHUNK;
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) {
        const int64_t j = base + k * RED_THREADS + threadIdx.x;
        if (j < n)
            acc += v[j];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(RED_THREADS)
k_sum_final(const double* __restrict__ part, int64_t n, double* out, int do_sqrt)
{
    __shared__ double s[RED_THREADS];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += RED_THREADS)
        acc += part[j];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = do_sqrt ? sqrt(s[0]) : s[0];
}

void sum_to(const double* v, int64_t n, double* part, double* out, bool do_sqrt, hipStream_t st)
{
    const int64_t nb = (n + RED_CHUNK - 1) / RED_CHUNK;
    if (nb == 0) {
        k_sum_final<<<1, RED_THREADS, 0, st>>>(part, 0, out, do_sqrt ? 1 : 0);
        return;
    }
    k_sum_partial<<<(unsigned)nb, RED_THREADS, 0, st>>>(v, n, part);
    k_sum_final<<<1, RED_THREADS, 0, st>>>(part, nb, out, do_sqrt ? 1 : 0);
}

size_t sum_partials(int64_t n) { return (size_t)((n + RED_CHUNK - 1) / RED_CHUNK + 1); }

static unsigned grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1)
        g = 1;
    if (g > 1 << 20)
        g = 1 << 20;
    return (unsigned)g;
}

// ------------------------------------------------------------------ launchers

template <typename T>
static void launch_interp(const Grid& g, int P, const ib_markers* m, const T* u, T* U,
                          hipStream_t st)
{
    if (m->nl == 0)
        return;
    const unsigned gb = grid_for(m->nl, 256);
    if (P == 3)
        k_interp_plain<T, 3><<<gb, 256, 0, st>>>(g, m->nl, m->x, m->y, m->z, u, U);
    else
        k_interp_plain<T, 4><<<gb, 256, 0, st>>>(g, m->nl, m->x, m->y, m->z, u, U);
}

template <typename T>
static void launch_spread(const Grid& g, int P, const ib_markers* m, const ib_buckets* b,
                          const T* F, T* f, T scale, int use_dv, hipStream_t st)
{
    if (g.ntiles == 0)
        return;
    const unsigned gt = (unsigned)g.ntiles;
    if (P == 3)
        k_spread_plain<T, 3><<<gt, TILE_CELLS, 0, st>>>(g, m->x, m->y, m->z, m->pid, m->dv,
                                                        b->perm, b->src_offs, b->src_idx, F, f,
                                                        scale, use_dv);
    else
        k_spread_plain<T, 4><<<gt, TILE_CELLS, 0, st>>>(g, m->x, m->y, m->z, m->pid, m->dv,
                                                        b->perm, b->src_offs, b->src_idx, F, f,
                                                        scale, use_dv);
}

void plain_interp(const Grid& g, int P, ib_prec prec, const ib_markers* m, const void* u,
                  void* U, hipStream_t st)
{
    if (prec == IB_F64)
        launch_interp<double>(g, P, m, (const double*)u, (double*)U, st);
    else
        launch_interp<float>(g, P, m, (const float*)u, (float*)U, st);
}

void plain_spread(const Grid& g, int P, ib_prec prec, const ib_markers* m, const ib_buckets* b,
                  const void* F, void* f, double scale, int use_dv, hipStream_t st)
{
    if (prec == IB_F64)
        launch_spread<double>(g, P, m, b, (const double*)F, (double*)f, scale, use_dv, st);
    else
        launch_spread<float>(g, P, m, b, (const float*)F, (float*)f, (float)scale, use_dv, st);
}

size_t field_elems(const Grid& g) { return (size_t)g.nbox * (size_t)g.bstride; }

size_t plain_workspace(const Grid& g, ib_prec prec, int64_t nl)
{
    const size_t s = prec == IB_F64 ? 8 : 4;
    Carver cv(nullptr, 0);
    cv.take<char>(s * 3 * nl);       // U
    cv.take<char>(s * 3 * nl);       // U^d
    cv.take<double>(nl);             // residual terms
    cv.take<double>(sum_partials(nl));
    cv.take<char>(s * field_elems(g));  // f when the caller passes none
    return cv.used;
}

template <typename T>
static int plain_loop(const Grid& g, int P, const ib_particles* p, const ib_markers* m,
                      const ib_buckets* b, int ns, double dt, const T* u0, T* ustar, T* f,
                      T* F, double* resid, T* Fhist, void* ws, size_t ws_bytes, hipStream_t st)
{
    const int64_t nl = m->nl;
    Carver cv(ws, ws_bytes);
    T* U = cv.take<T>(3 * nl);
    T* Ud = cv.take<T>(3 * nl);
    double* e2 = cv.take<double>(nl);
    double* part = cv.take<double>(sum_partials(nl));
    T* fws = cv.take<T>(field_elems(g));
    if (!cv.ok())
        return IB_EWORKSPACE;
    if (!f)
        f = fws;
    const unsigned gm = grid_for(nl, 256);
    const unsigned gc = grid_for((int64_t)g.nbox * g.box * g.box * g.box, 256);
    desired_velocity(p, m, sizeof(T) == 8 ? IB_F64 : IB_F32, Ud, st);
    if (nl > 0)
        k_zero_vec<T><<<gm, 256, 0, st>>>(3 * nl, F);
    if (ns == 0) {
        k_correct<T><<<gc, 256, 0, st>>>(g, dt, u0, nullptr, ustar);
        k_zero_field<T><<<gc, 256, 0, st>>>(g, f);
    }
    for (int mi = 1; mi <= ns; ++mi) {
        const T* uprev = (mi == 1) ? u0 : ustar;
        launch_interp<T>(g, P, m, uprev, U, st);
        if (nl > 0)
            k_force_update<T><<<gm, 256, 0, st>>>(nl, dt, Ud, U, F, m->pid, m->dv,
                                                  resid ? e2 : nullptr);
        if (resid)
            sum_to(e2, nl, part, resid + (mi - 1), true, st);
        if (Fhist && nl > 0)
            k_copy_vec<T><<<gm, 256, 0, st>>>(3 * nl, F, Fhist + (int64_t)(mi - 1) * 3 * nl);
        launch_spread<T>(g, P, m, b, F, f, T(1), 1, st);
        k_correct<T><<<gc, 256, 0, st>>>(g, dt, u0, f, ustar);
    }
    if (resid) {
        launch_interp<T>(g, P, m, ns ? ustar : u0, U, st);
        if (nl > 0)
            k_resid_only<T><<<gm, 256, 0, st>>>(nl, Ud, U, m->pid, m->dv, e2);
        sum_to(e2, nl, part, resid + ns, true, st);
    }
    PoisonSet ps;
    ps.field[0] = ustar;
    ps.field[1] = f;
    ps.vec[0] = F;
    ps.nvec[0] = 3 * nl;
    ps.vec[1] = Fhist;
    ps.nvec[1] = 3 * nl * ns;
    ps.dvec[0] = resid;
    ps.ndvec[0] = ns + 1;
    poison_if_flagged(b->flag, g, sizeof(T) == 8 ? IB_F64 : IB_F32, ps, st);
    return launch_status();
}

int plain_multidirect(const Grid& g, int P, ib_prec prec, const ib_particles* p,
                      const ib_markers* m, const ib_buckets* b, int ns, double dt,
                      const void* u0, void* ustar, void* f, void* F, double* resid, void* Fhist,
                      void* ws, size_t ws_bytes, hipStream_t st)
{
    if (prec == IB_F64)
        return plain_loop<double>(g, P, p, m, b, ns, dt, (const double*)u0, (double*)ustar,
                                  (double*)f, (double*)F, resid, (double*)Fhist, ws, ws_bytes,
                                  st);
    return plain_loop<float>(g, P, p, m, b, ns, dt, (const float*)u0, (float*)ustar, (float*)f,
                             (float*)F, resid, (float*)Fhist, ws, ws_bytes, st);
}

}  // namespace ibx

using namespace ibx;

extern "C" int ib_interp(const ib_level* lv, const ib_markers* m, ib_delta delta, ib_prec prec,
                         const void* u, void* U, void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!m || (delta != IB_DELTA3 && delta != IB_DELTA4) || (prec != IB_F32 && prec != IB_F64) ||
        m->nl < 0 || (m->nl > 0 && (!m->x || !m->y || !m->z || !u || !U)))
        return IB_EINVAL;
    plain_interp(make_grid(lv), (int)delta, prec, m, u, U, (hipStream_t)stream);
    return launch_status();
}

extern "C" int ib_spread(const ib_level* lv, const ib_markers* m, const ib_buckets* b,
                         ib_delta delta, ib_prec prec, const void* F, void* f, void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!m || !b || !f || (delta != IB_DELTA3 && delta != IB_DELTA4) ||
        (prec != IB_F32 && prec != IB_F64) || m->nl < 0 || !b->src_offs ||
        (m->nl > 0 && (!m->x || !m->y || !m->z || !m->pid || !m->dv || !F || !b->perm ||
                       !b->src_idx)))
        return IB_EINVAL;
    const Grid g = make_grid(lv);
    plain_spread(g, (int)delta, prec, m, b, F, f, 1.0, 1, (hipStream_t)stream);
    PoisonSet ps;
    ps.field[0] = f;
    poison_if_flagged(b->flag, g, prec, ps, (hipStream_t)stream);
    return launch_status();
}
