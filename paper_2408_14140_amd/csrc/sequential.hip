// sequential.hip -- the particle-by-particle order of the coupling loop.
//
// Sec. 3.1 (the remarks after Algorithm 1) has every particle run the N_s
// loop in turn, on the velocity field its predecessors left, with the forces
// of all particles adding up in f.  Two particles whose delta-kernel supports
// share no cell do not see each other inside a loop, so they commute.  Conflict
// levels order the rest: level(j) = 0 when no earlier particle's support may
// meet j's, else 1 + the largest level among those that may.  Running the
// levels in increasing order, each level as one batched loop over all of its
// particles (disjoint supports: the batched Jacobi sum equals the one-by-one
// sweep), keeps every conflicting pair in index order and so reproduces the
// particle-by-particle result up to rounding.
//
// Support test (conservative): every stencil cell centre lies within P/2 cells
// of its marker on each axis, so two supports can share a cell only when two
// markers are within sqrt(3) P h; markers lie within D/2 of their centroid.
// The test uses the minimum-image centroid distance < (D_i + D_j)/2 + 2 P h.
// A pair flagged without a shared cell only adds an ordering constraint.
#include <vector>

#include "paths.h"

namespace ibx {

constexpr int LV_WAVES = 4;
constexpr int MAX_LEVELS = SEQ_MAX_LEVELS;
constexpr int ORDER_THREADS = 1024;

__global__ void k_fill_i32(int64_t n, int32_t* a, int32_t v)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = v;
}

// One relaxation: lout[j] = 1 + max(lin[i] : i < j, supports may meet), or 0.
// One wavefront per particle; lanes stride over the earlier particles.  The
// map is monotone and starts from zero, so repeating it reaches the longest
// conflict chain ending at each particle.
__global__ void __launch_bounds__(64 * LV_WAVES)
k_levels_step(int32_t np, const double* __restrict__ xc, const double* __restrict__ d,
              double reach, double L0, double L1, double L2, const int32_t* __restrict__ lin,
              int32_t* __restrict__ lout, int32_t* __restrict__ changed)
{
    const int j = blockIdx.x * LV_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= np)
        return;
    const double L[3] = {L0, L1, L2};
    const double xj[3] = {xc[3 * j], xc[3 * j + 1], xc[3 * j + 2]};
    const double dj = d[j];
    int best = -1;
    // explicitly rounded operations (no contraction): the test is an integer
    // decision that the same FP64 expression must reproduce anywhere
    for (int i = lane; i < j; i += 64) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double del = __dsub_rn(xc[3 * i + c], xj[c]);
            if (L[c] > 0.0) {
                const double k = floor(__dadd_rn(__ddiv_rn(del, L[c]), 0.5));
                del = __dsub_rn(del, __dmul_rn(L[c], k));
            }
            r2 = __dadd_rn(r2, __dmul_rn(del, del));
        }
        const double lim = __dadd_rn(__dmul_rn(0.5, __dadd_rn(d[i], dj)), reach);
        if (r2 < __dmul_rn(lim, lim))
            best = max(best, lin[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        best = max(best, __shfl_xor(best, o));
    if (lane == 0) {
        const int lvl = best + 1;
        lout[j] = lvl;
        if (lvl != lin[j])
            changed[0] = 1;
    }
}

// out[0] = 1 + max level (the number of levels).
__global__ void __launch_bounds__(1024)
k_count_levels(int32_t np, const int32_t* __restrict__ lvl, int32_t* __restrict__ out)
{
    __shared__ int32_t red[1024];
    int m = -1;
    for (int j = threadIdx.x; j < np; j += 1024)
        m = max(m, lvl[j]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = red[0] + 1;
}

// Particles in (level, index) order, the first particle of each level and the
// marker offsets in that order.  One workgroup.  err[0] = 1 (and nothing else
// written) when a level is out of range or offs is not a partition of
// [0, nl) into consecutive runs.
__global__ void __launch_bounds__(ORDER_THREADS)
k_level_order(int32_t np, const int32_t* __restrict__ level, int32_t nlev,
              const int64_t* __restrict__ offs, int64_t nl, int32_t* __restrict__ pord,
              int32_t* __restrict__ loffs, int64_t* __restrict__ noffs, int32_t* __restrict__ err)
{
    __shared__ int32_t cnt[MAX_LEVELS];
    __shared__ int32_t chunk[ORDER_THREADS];
    __shared__ int64_t part[ORDER_THREADS];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0)
        bad = (offs[0] != 0 || offs[np] != nl) ? 1 : 0;
    __syncthreads();
    for (int j = t; j < np; j += ORDER_THREADS) {
        const int lj = level[j];
        if (lj < 0 || lj >= nlev || offs[j + 1] < offs[j])
            bad = 1;
    }
    for (int c = t; c < nlev; c += ORDER_THREADS)
        cnt[c] = 0;
    __syncthreads();
    if (bad) {
        if (t == 0)
            err[0] = 1;
        return;
    }
    for (int j = t; j < np; j += ORDER_THREADS)
        atomicAdd(&cnt[level[j]], 1);
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int c = 0; c < nlev; ++c) {
            const int v = cnt[c];
            cnt[c] = run;
            loffs[c] = run;
            run += v;
        }
        loffs[nlev] = run;
        err[0] = 0;
    }
    __syncthreads();
    // stable scatter: rank within the chunk among equal levels, chunk by chunk
    for (int b0 = 0; b0 < np; b0 += ORDER_THREADS) {
        const int j = b0 + t;
        const int lj = j < np ? level[j] : -1;
        chunk[t] = lj;
        __syncthreads();
        if (j < np) {
            int r = 0;
            for (int q = 0; q < t; ++q)
                r += chunk[q] == lj;
            pord[cnt[lj] + r] = j;
        }
        __syncthreads();
        if (j < np)
            atomicAdd(&cnt[lj], 1);
        __syncthreads();
    }
    // marker offsets in the new order: inclusive scan of the counts
    int64_t carry = 0;
    if (t == 0)
        noffs[0] = 0;
    for (int b0 = 0; b0 < np; b0 += ORDER_THREADS) {
        const int k = b0 + t;
        int64_t v = 0;
        if (k < np) {
            const int p = pord[k];
            v = offs[p + 1] - offs[p];
        }
        part[t] = v;
        __syncthreads();
        for (int o = 1; o < ORDER_THREADS; o <<= 1) {
            const int64_t add = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        if (k < np)
            noffs[k + 1] = carry + part[t];
        carry += part[ORDER_THREADS - 1];
        __syncthreads();
    }
}

__global__ void k_gather_particles(int32_t np, const int32_t* __restrict__ pord,
                                   const double* __restrict__ xc, const double* __restrict__ d,
                                   const double* __restrict__ up, const double* __restrict__ om,
                                   const double* __restrict__ dv, double* __restrict__ xr,
                                   double* __restrict__ dr, double* __restrict__ upr,
                                   double* __restrict__ omr, double* __restrict__ dvr)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np)
        return;
    const int p = pord[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xr[3 * k + c] = xc[3 * p + c];
        upr[3 * k + c] = up[3 * p + c];
        omr[3 * k + c] = om[3 * p + c];
    }
    dr[k] = d[p];
    dvr[k] = dv[p];
}

// Markers of the k-th particle in level order copied to their new run;
// mmap[new] = old marker index.
__global__ void k_gather_markers(int32_t np, const int32_t* __restrict__ pord,
                                 const int64_t* __restrict__ offs,
                                 const int64_t* __restrict__ noffs, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ z,
                                 double* __restrict__ xr, double* __restrict__ yr,
                                 double* __restrict__ zr, int32_t* __restrict__ pidr,
                                 int32_t* __restrict__ mmap)
{
    for (int k = blockIdx.x; k < np; k += gridDim.x) {
        const int p = pord[k];
        const int64_t s0 = offs[p], cnt = offs[p + 1] - s0, d0 = noffs[k];
        for (int64_t q = threadIdx.x; q < cnt; q += blockDim.x) {
            xr[d0 + q] = x[s0 + q];
            yr[d0 + q] = y[s0 + q];
            zr[d0 + q] = z[s0 + q];
            pidr[d0 + q] = k;
            mmap[d0 + q] = (int32_t)(s0 + q);
        }
    }
}

template <typename T>
__global__ void k_scatter_F(int64_t nl, const int32_t* __restrict__ mmap,
                            const T* __restrict__ Fr, T* __restrict__ F)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nl)
        return;
    const int64_t l = mmap[q];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        F[3 * l + c] = Fr[3 * q + c];
}

__global__ void k_or_flags(const int32_t* __restrict__ src, int32_t* __restrict__ dst)
{
    if (threadIdx.x < 2 && src[threadIdx.x])
        dst[threadIdx.x] = 1;
}

struct SeqWs {
    double *xc, *d, *up, *om, *dv;
    int32_t *pord, *loffs, *err, *anyflag;
    int64_t* noffs;
    double *x, *y, *z;
    int32_t *pid, *mmap;
    char* F;
    ib_buckets b;
    void* bws;
    size_t bws_bytes;
    void* lws;
    size_t lws_bytes;
};

static SeqWs carve_seq(const ib_level* lv, const Grid& g, ib_prec prec, int32_t np, int64_t nl,
                       const BatchedCfg& cfg, void* ws, size_t bytes, size_t* need)
{
    Carver cv(ws, bytes);
    SeqWs w;
    w.xc = cv.take<double>(3 * (size_t)np);
    w.d = cv.take<double>(np);
    w.up = cv.take<double>(3 * (size_t)np);
    w.om = cv.take<double>(3 * (size_t)np);
    w.dv = cv.take<double>(np);
    w.pord = cv.take<int32_t>(np);
    w.loffs = cv.take<int32_t>((size_t)np + 1);
    w.err = cv.take<int32_t>(1);
    w.anyflag = cv.take<int32_t>(2);
    w.noffs = cv.take<int64_t>((size_t)np + 1);
    w.x = cv.take<double>(nl);
    w.y = cv.take<double>(nl);
    w.z = cv.take<double>(nl);
    w.pid = cv.take<int32_t>(nl);
    w.mmap = cv.take<int32_t>(nl);
    w.F = cv.take<char>(3 * (size_t)nl * (prec == IB_F64 ? 8 : 4));
    w.b.cell = cv.take<int32_t>(nl);
    w.b.tileid = cv.take<int32_t>(nl);
    w.b.base = cv.take<int32_t>(3 * (size_t)nl);
    w.b.perm = cv.take<int32_t>(nl);
    w.b.tile_offs = cv.take<int32_t>((size_t)g.ntiles + 1);
    w.b.src_offs = cv.take<int32_t>((size_t)g.ntiles + 1);
    w.b.src_cap = 8 * nl;
    w.b.src_idx = cv.take<int32_t>((size_t)w.b.src_cap);
    w.b.flag = cv.take<int32_t>(2);
    w.bws_bytes = ib_bucket_workspace(lv, nl);
    w.bws = cv.take<char>(w.bws_bytes);
    BatchedCfg c = cfg;
    c.bw = 64;  // the narrowest width needs the most work items
    w.lws_bytes = batched_workspace(g, prec, nl, c);
    w.lws = cv.take<char>(w.lws_bytes);
    *need = cv.used;
    return w;
}

size_t sequential_workspace(const ib_level* lv, const Grid& g, ib_prec prec, int32_t np,
                            int64_t nl, const BatchedCfg& cfg)
{
    size_t need = 0;
    carve_seq(lv, g, prec, np, nl, cfg, nullptr, 0, &need);
    return need;
}

static int hip_ok(hipError_t e)
{
    if (e != hipSuccess) {
        set_hip_error(e);
        return IB_EHIP;
    }
    return IB_OK;
}

int sequential_multidirect(const ib_level* lv, const Grid& g, int P, ib_prec prec,
                           const BatchedCfg& cfg, const ib_particles* p, const ib_markers* m,
                           int ns, double dt, const int32_t* level, int32_t nlevels,
                           const void* u0, void* ustar, void* f, void* F, int32_t* flag,
                           void* ws, size_t ws_bytes, hipStream_t st)
{
    const int32_t np = p->np;
    const int64_t nl = m->nl;
    size_t need = 0;
    carve_seq(lv, g, prec, np, nl, cfg, nullptr, 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    SeqWs w = carve_seq(lv, g, prec, np, nl, cfg, ws, ws_bytes, &need);
    if (flag)
        k_fill_i32<<<1, 64, 0, st>>>(2, flag, 0);
    k_fill_i32<<<1, 64, 0, st>>>(2, w.anyflag, 0);
    if (nl == 0) {
        // no marker: one empty loop writes ustar = u0 and f = 0
        ib_markers me = *m;
        me.nl = 0;
        int rc = ib_bucket(lv, &me, (ib_delta)P, &w.b, w.bws, w.bws_bytes, st);
        if (rc)
            return rc;
        return batched_multidirect(g, P, prec, cfg, p, &me, &w.b, ns, dt, u0, ustar, f, F,
                                   nullptr, nullptr, w.lws, w.lws_bytes, st, 0);
    }
    k_level_order<<<1, ORDER_THREADS, 0, st>>>(np, level, nlevels, m->offs, nl, w.pord, w.loffs,
                                               w.noffs, w.err);
    int rc = launch_status();
    if (rc)
        return rc;
    std::vector<int32_t> loffs((size_t)nlevels + 1);
    std::vector<int64_t> noffs((size_t)np + 1);
    int32_t err = 1;
    rc = hip_ok(hipMemcpyAsync(&err, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (!rc)
        rc = hip_ok(hipStreamSynchronize(st));
    if (rc)
        return rc;
    if (err)
        return IB_EINVAL;
    rc = hip_ok(hipMemcpyAsync(loffs.data(), w.loffs, sizeof(int32_t) * loffs.size(),
                               hipMemcpyDeviceToHost, st));
    if (!rc)
        rc = hip_ok(hipMemcpyAsync(noffs.data(), w.noffs, sizeof(int64_t) * noffs.size(),
                                   hipMemcpyDeviceToHost, st));
    if (!rc)
        rc = hip_ok(hipStreamSynchronize(st));
    if (rc)
        return rc;
    if (loffs[nlevels] != np || noffs[np] != nl)
        return IB_EINVAL;
    k_gather_particles<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(
        np, w.pord, p->xc, p->d, p->up, p->om, m->dv, w.xc, w.d, w.up, w.om, w.dv);
    k_gather_markers<<<(unsigned)(np < 65535 ? np : 65535), 256, 0, st>>>(
        np, w.pord, m->offs, w.noffs, m->x, m->y, m->z, w.x, w.y, w.z, w.pid, w.mmap);
    rc = launch_status();
    if (rc)
        return rc;
    ib_particles pr;
    pr.np = np;
    pr.xc = w.xc;
    pr.d = w.d;
    pr.up = w.up;
    pr.om = w.om;
    const size_t es = prec == IB_F64 ? 8 : 4;
    const void* uin = u0;
    int first = 1;
    for (int c = 0; c < nlevels; ++c) {
        const int64_t n0 = noffs[loffs[c]], n1 = noffs[loffs[c + 1]];
        if (n1 == n0)
            continue;
        ib_markers mc;
        mc.nl = n1 - n0;
        mc.offs = w.noffs + loffs[c];
        mc.x = w.x + n0;
        mc.y = w.y + n0;
        mc.z = w.z + n0;
        mc.pid = w.pid + n0;
        mc.dv = w.dv;
        rc = ib_bucket(lv, &mc, (ib_delta)P, &w.b, w.bws, w.bws_bytes, st);
        if (rc)
            return rc;
        if (flag)
            k_or_flags<<<1, 64, 0, st>>>(w.b.flag, flag);
        k_or_flags<<<1, 64, 0, st>>>(w.b.flag, w.anyflag);
        rc = batched_multidirect(g, P, prec, cfg, &pr, &mc, &w.b, ns, dt, uin, ustar, f,
                                 w.F + 3 * n0 * es, nullptr, nullptr, w.lws, w.lws_bytes, st,
                                 first ? 0 : 1);
        if (rc)
            return rc;
        uin = ustar;
        first = 0;
    }
    const unsigned gm = (unsigned)((nl + 255) / 256);
    if (prec == IB_F64)
        k_scatter_F<double><<<gm, 256, 0, st>>>(nl, w.mmap, (const double*)w.F, (double*)F);
    else
        k_scatter_F<float><<<gm, 256, 0, st>>>(nl, w.mmap, (const float*)w.F, (float*)F);
    // a flagged level leaves every output NaN, not only its own markers' F
    PoisonSet ps;
    ps.field[0] = ustar;
    ps.field[1] = f;
    ps.vec[0] = F;
    ps.nvec[0] = 3 * nl;
    poison_if_flagged(w.anyflag, g, prec, ps, st);
    return launch_status();
}

}  // namespace ibx

using namespace ibx;

extern "C" size_t ib_levels_workspace(int32_t np)
{
    if (np < 0)
        return 0;
    Carver cv(nullptr, 0);
    cv.take<int32_t>(np);
    cv.take<int32_t>(2);
    return cv.used;
}

extern "C" int ib_particle_levels(const ib_level* lv, const ib_particles* p, ib_delta delta,
                                  int32_t* level, int32_t* nlevels, void* ws, size_t ws_bytes,
                                  void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!p || p->np < 0 || !nlevels || (delta != IB_DELTA3 && delta != IB_DELTA4))
        return IB_EINVAL;
    const int32_t np = p->np;
    if (np == 0) {
        *nlevels = 0;
        return IB_OK;
    }
    if (!p->xc || !p->d || !level)
        return IB_EINVAL;
    if (!ws || ws_bytes < ib_levels_workspace(np))
        return IB_EWORKSPACE;
    Carver cv(ws, ws_bytes);
    int32_t* alt = cv.take<int32_t>(np);
    int32_t* flag = cv.take<int32_t>(2);
    hipStream_t st = (hipStream_t)stream;
    double L[3];
    for (int a = 0; a < 3; ++a)
        L[a] = lv->periodic[a] ? lv->n[a] * lv->h : 0.0;
    const double reach = 2.0 * (double)delta * lv->h;
    const unsigned gp = (unsigned)((np + 255) / 256);
    const unsigned gl = (unsigned)((np + LV_WAVES - 1) / LV_WAVES);
    k_fill_i32<<<gp, 256, 0, st>>>(np, level, 0);
    int32_t* a = level;
    int32_t* b = alt;
    // at most np relaxations: a chain of conflicts is at most np long
    for (int32_t it = 0; it <= np; ++it) {
        k_fill_i32<<<1, 64, 0, st>>>(1, flag, 0);
        k_levels_step<<<gl, 64 * LV_WAVES, 0, st>>>(np, p->xc, p->d, reach, L[0], L[1], L[2], a,
                                                   b, flag);
        rc = launch_status();
        if (rc)
            return rc;
        int32_t changed = 0;
        rc = hip_ok(hipMemcpyAsync(&changed, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        if (!rc)
            rc = hip_ok(hipStreamSynchronize(st));
        if (rc)
            return rc;
        int32_t* t = a;
        a = b;
        b = t;
        if (!changed)
            break;
    }
    if (a != level) {
        rc = hip_ok(hipMemcpyAsync(level, a, sizeof(int32_t) * (size_t)np,
                                   hipMemcpyDeviceToDevice, st));
        if (rc)
            return rc;
    }
    k_count_levels<<<1, 1024, 0, st>>>(np, level, flag + 1);
    rc = launch_status();
    if (rc)
        return rc;
    int32_t nlev = 0;
    rc = hip_ok(hipMemcpyAsync(&nlev, flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (!rc)
        rc = hip_ok(hipStreamSynchronize(st));
    if (rc)
        return rc;
    *nlevels = nlev;
    return IB_OK;
}
