// rigid.hip -- the particle side of a time step (Sec. 3.2; Step 4 of
// Sec. 3.1): rigid-body update of the spheres, rigid advection of their
// markers and the repulsive collision force.  One thread per particle or per
// marker; FP64 throughout.
#include "ibx_internal.h"

namespace ibx {

// Eqs. (particle1), (particle2) with their right-hand sides at the half
// step: marker force F^{n+1/2} of Algorithm 1 (raw sums S_F, S_T from the
// per-particle reductions), volume integrals differenced over dt, buoyancy
// and an optional collision force and torque.  V_p = pi D^3/6, I_p =
// rho_p V_p D^2/10.  Prescribed particles keep U and W.  Centroid by
// Eq. (pr2): X^{n+1} = X^n + dt/2 (U^n + U^{n+1}).
__global__ void __launch_bounds__(256)
k_rigid_update(int32_t np, const double* __restrict__ xc, const double* __restrict__ d,
               const double* __restrict__ up, const double* __restrict__ om,
               const double* __restrict__ rho_p, const double* __restrict__ s0,
               const double* __restrict__ s1, const double* __restrict__ Fc,
               const double* __restrict__ Tc, const int32_t* __restrict__ prescribed,
               double rho_f, double g0, double g1, double g2, double dt,
               double* __restrict__ up1, double* __restrict__ om1, double* __restrict__ xc1)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    const double D = d[p];
    const double Vp = 3.14159265358979323846 * D * D * D / 6.0;
    const double mass = rho_p[p] * Vp;
    const double Ip = mass * D * D / 10.0;
    const double g[3] = {g0, g1, g2};
    const bool fixed = prescribed && prescribed[p];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double un = up[3 * p + c], wn = om[3 * p + c];
        double u = un, w = wn;
        if (!fixed) {
            const double force = -rho_f * s0[12 * p + c] +
                                 rho_f * (s1[12 * p + 6 + c] - s0[12 * p + 6 + c]) / dt +
                                 (rho_p[p] - rho_f) * Vp * g[c] + (Fc ? Fc[3 * p + c] : 0.0);
            const double torque = -rho_f * s0[12 * p + 3 + c] +
                                  rho_f * (s1[12 * p + 9 + c] - s0[12 * p + 9 + c]) / dt +
                                  (Tc ? Tc[3 * p + c] : 0.0);
            u = un + dt * force / mass;
            w = wn + dt * torque / Ip;
        }
        up1[3 * p + c] = u;
        om1[3 * p + c] = w;
        xc1[3 * p + c] = xc[3 * p + c] + 0.5 * dt * (un + u);
    }
}

// Eq. (x) for a rigid body: X^{n+1} = X_r^{n+1} + Q R^n with Q the rotation
// by |W| dt about W, W = (W^n + W^{n+1})/2 (Rodrigues' formula).  In place
// when the output arrays are the input ones.
__global__ void __launch_bounds__(256)
k_advect_markers(int64_t nl, const double* x, const double* y, const double* z,
                 const int32_t* __restrict__ pid, const double* __restrict__ xc_n,
                 const double* __restrict__ xc_np1, const double* __restrict__ om_n,
                 const double* __restrict__ om_np1, double dt, double* xn, double* yn,
                 double* zn)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    const int p = pid[l];
    const double R[3] = {x[l] - xc_n[3 * p], y[l] - xc_n[3 * p + 1], z[l] - xc_n[3 * p + 2]};
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        w[c] = 0.5 * (om_n[3 * p + c] + om_np1[3 * p + c]);
    const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double o[3] = {R[0], R[1], R[2]};
    if (wn > 0.0) {
        const double k[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
        double st, ct;
        sincos(wn * dt, &st, &ct);
        const double kxr[3] = {k[1] * R[2] - k[2] * R[1], k[2] * R[0] - k[0] * R[2],
                               k[0] * R[1] - k[1] * R[0]};
        const double kdr = k[0] * R[0] + k[1] * R[1] + k[2] * R[2];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            o[c] = R[c] * ct + kxr[c] * st + k[c] * kdr * (1.0 - ct);
    }
    xn[l] = xc_np1[3 * p] + o[0];
    yn[l] = xc_np1[3 * p + 1] + o[1];
    zn[l] = xc_np1[3 * p + 2] + o[2];
}

// ---------------------------------------------------------------- collisions
// Eq. (DKT_model): F_c,ij = -(m |g| / eps_c) ((|delta| - D_c)/h)^2 delta/|delta|
// for |delta| < D_c = R_i + R_j + h, delta = X_j - X_i by the minimum image on
// periodic axes, m the mean of the two masses; the force on particle i is the
// sum over its partners j.  Partners are found through bins: cubes of an edge
// that is a multiple of 8 cells (a whole number of tiles) and no shorter than
// the largest interaction distance D_max + h (plus a cell), so every partner
// of a particle sits in one of the bins around its own (every bin is at least
// that wide; the last bin along an axis takes the remainder).  The bin edge
// follows from D_max on the device, so nothing is read back.  The particles
// are put in bin order (ascending index within a bin: by counting up to
// CS_MAX_NP particles, else by a stable radix sort), and each particle sums
// its partners bin by bin in a fixed order: the result does not depend on
// scheduling, and the two orderings give the same bits.

// Bins per axis are capped at 40 (64000 bins), so a bin key has 16 bits and
// sorts in two radix passes; a capped axis gets wider bins, still correct.
constexpr int CB_MAX_AXIS = 40;
constexpr int CB_MAX_BINS = CB_MAX_AXIS * CB_MAX_AXIS * CB_MAX_AXIS;

struct CollBins {
    int32_t edge[3];   // bin edge in cells per axis
    int32_t nb[3];     // bins per axis
};

constexpr int CB_THREADS = 1024;

// D_max over the particles by one workgroup of NT threads, then the bin
// geometry: every thread of the workgroup gets it.
template <int NT>
__device__ CollBins block_coll_bins(int32_t np, const double* __restrict__ d, double h, int n0,
                                    int n1, int n2)
{
    __shared__ double mx[NT / 64];
    __shared__ CollBins sb;
    double m = 0.0;
    // eight loads in flight per thread
    for (int64_t base = 0; base < np; base += 8 * NT) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = base + k * NT + threadIdx.x;
            v[k] = i < np ? d[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            m = fmax(m, v[k]);
    }
    for (int o = 32; o > 0; o >>= 1)
        m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0)
        mx[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NT / 64; ++w)
            m = fmax(m, mx[w]);
        // largest D_c = D_max + h in cells, one cell more for the rounding
        // of a centroid's cell, then whole tiles
        double ec = ceil((m + h) / h) + 1.0;
        if (!(ec < 1.0e9))
            ec = 1.0e9;
        int64_t e = (int64_t)ec;
        e = (e + TILE - 1) / TILE * TILE;
        const int n[3] = {n0, n1, n2};
        for (int a = 0; a < 3; ++a) {
            int ea = e < n[a] ? (int)e : n[a];
            if (n[a] / ea > CB_MAX_AXIS)  // wider bins: at most CB_MAX_AXIS of them
                ea = ((n[a] + CB_MAX_AXIS - 1) / CB_MAX_AXIS + TILE - 1) / TILE * TILE;
            sb.edge[a] = ea;
            sb.nb[a] = n[a] / ea > 1 ? n[a] / ea : 1;
        }
    }
    __syncthreads();
    return sb;
}

__global__ void __launch_bounds__(CB_THREADS)
k_coll_bins(int32_t np, const double* __restrict__ d, double h, int n0, int n1, int n2,
            CollBins* __restrict__ cb)
{
    const CollBins b = block_coll_bins<CB_THREADS>(np, d, h, n0, n1, n2);
    if (threadIdx.x == 0)
        *cb = b;
}

// Bin along each axis of a centroid x from its cell floor((x - lo)/h), the
// quotient taken as a product with 1/h (binning needs only to agree with
// itself, and the bins carry a cell of margin); wrapped on a periodic axis,
// clamped on a bounded one; a non-finite centroid lands in bin 0 and meets no
// partner.
__device__ inline void coll_bin(const Grid& g, const CollBins& cb, const double* x, int* b)
{
    const double inv_h = 1.0 / g.h;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double t = floor((x[a] - g.lo[a]) * inv_h);
        const int n = g.n[a];
        int c;
        if (t >= 0.0 && t < n) {
            c = (int)t;
        } else if (g.periodic[a]) {
            const double u = t - n * floor(t / n);
            c = u >= 0.0 && u < n ? (int)u : 0;
        } else {
            c = t >= n ? n - 1 : 0;
        }
        const int q = c / cb.edge[a];
        b[a] = q < cb.nb[a] ? q : cb.nb[a] - 1;
    }
}

// Mass rho V of a sphere of diameter D, V = pi D^3/6.
__device__ inline double sphere_mass(double rho, double D)
{
    return rho * 3.14159265358979323846 * D * D * D / 6.0;
}

// A particle in bin order: centroid, diameter, mass, index.
struct CollPart {
    double x, y, z, d, m;
    int32_t id, pad;
};

__device__ inline void coll_gather(int32_t j, const double* __restrict__ xc,
                                   const double* __restrict__ d,
                                   const double* __restrict__ rho_p, CollPart* __restrict__ out)
{
    CollPart c;
    c.x = xc[3 * j];
    c.y = xc[3 * j + 1];
    c.z = xc[3 * j + 2];
    c.d = d[j];
    c.m = sphere_mass(rho_p[j], c.d);
    c.id = j;
    c.pad = 0;
    *out = c;
}

__global__ void k_coll_keys(int32_t np, Grid g, const double* __restrict__ xc,
                            const CollBins* __restrict__ cbp, int32_t* __restrict__ keys,
                            int32_t* __restrict__ vals)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np)
        return;
    const CollBins cb = *cbp;
    int b[3];
    coll_bin(g, cb, xc + 3 * i, b);
    keys[i] = b[0] + cb.nb[0] * (b[1] + cb.nb[1] * b[2]);
    vals[i] = i;
}

// The particles in sorted order (radix path).
__global__ void k_coll_gather(int32_t np, const int32_t* __restrict__ sorted,
                              const double* __restrict__ xc, const double* __restrict__ d,
                              const double* __restrict__ rho_p, CollPart* __restrict__ ps)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < np)
        coll_gather(sorted[q], xc, d, rho_p, ps + q);
}

// Up to CS_MAX_NP particles the set-up is one launch.  Every workgroup finds
// the bin geometry and the words bin << CS_IDX_BITS | index of all particles
// (in LDS); the words are distinct, so a particle's place in the stable sort
// by bin (bins ascending, ascending index within a bin) is the number of
// smaller words.  Each particle writes itself to its place, and the first
// particle of a bin writes the bin offsets (offs[b] = first place with bin
// >= b) from the bin after the previous occupied one up to its own; the last
// particle writes them up to the bin count.
constexpr int CS_IDX_BITS = 13;
constexpr int CS_MAX_NP = 1 << CS_IDX_BITS;
constexpr int CR_THREADS = 256;
constexpr int CR_WAVES = CR_THREADS / 64;

// A workgroup ranks 64 particles (one per lane); its wavefronts count over
// quarters of the words and add their counts up in LDS.
__global__ void __launch_bounds__(CR_THREADS)
k_coll_rank(int32_t np, Grid g, const double* __restrict__ xc, const double* __restrict__ d,
            const double* __restrict__ rho_p, CollBins* __restrict__ cbo,
            CollPart* __restrict__ ps, int32_t* __restrict__ offs)
{
    __shared__ uint32_t s[CS_MAX_NP];
    __shared__ int pr[CR_WAVES][64];
    __shared__ uint32_t pm[CR_WAVES][64];
    const CollBins cb = block_coll_bins<CR_THREADS>(np, d, g.h, g.n[0], g.n[1], g.n[2]);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *cbo = cb;
    for (int i = threadIdx.x; i < np; i += CR_THREADS) {
        int b[3];
        coll_bin(g, cb, xc + 3 * i, b);
        s[i] = ((uint32_t)(b[0] + cb.nb[0] * (b[1] + cb.nb[1] * b[2])) << CS_IDX_BITS) |
               (uint32_t)i;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 64 + lane;
    const uint32_t wi = i < np ? s[i] : 0u;
    const int chunk = (np + CR_WAVES - 1) / CR_WAVES;
    const int q1 = min(np, (wv + 1) * chunk);
    int r = 0;
    uint32_t mw = 0;  // the largest smaller word, valid when r > 0
#pragma unroll 8
    for (int q = wv * chunk; q < q1; ++q) {
        const uint32_t w = s[q];  // the same word on every lane: a broadcast read
        const bool lt = w < wi;
        r += lt;
        mw = lt && w > mw ? w : mw;
    }
    pr[wv][lane] = r;
    pm[wv][lane] = mw;
    __syncthreads();
    if (wv != 0 || i >= np)
        return;
    r = 0;
    bool any = false;
    for (int k = 0; k < CR_WAVES; ++k) {
        if (pr[k][lane] > 0) {
            mw = any && mw > pm[k][lane] ? mw : pm[k][lane];
            any = true;
        }
        r += pr[k][lane];
    }
    coll_gather(i, xc, d, rho_p, ps + r);
    const int key = (int)(wi >> CS_IDX_BITS);
    const int prev = r > 0 ? (int)(mw >> CS_IDX_BITS) : -1;
    for (int bb = prev + 1; bb <= key; ++bb)
        offs[bb] = r;
    if (r == np - 1) {
        const int nbins = cb.nb[0] * cb.nb[1] * cb.nb[2];
        for (int bb = key + 1; bb <= nbins; ++bb)
            offs[bb] = np;
    }
}

// One wavefront per particle, taken in bin order, over the bins around its
// own: offsets -1, 0, 1 per axis (0, 1 on a periodic axis of two bins, 0 on
// an axis of one bin, so no bin is visited twice), in the order z, y, x with x
// fastest.  Lane k < 27 reads the range of the k-th bin, a wave scan joins the
// ranges into one candidate list (bin after bin, ascending index within a
// bin), and lane k takes the entries k, k + 64, ...; the lanes' partial sums
// then meet in a fixed butterfly.  The minimum image skips its division where
// |delta| is below a quarter period (the shift is zero there).  The force of
// a pair is formed as s delta with s = m (|g|/eps_c) q^2 / |delta|,
// q = (|delta| - D_c)/h: one square root and one division per pair in reach.
constexpr int CW_WAVES = 4;

__global__ void __launch_bounds__(64 * CW_WAVES)
k_collide_bins(int32_t np, Grid g, const CollPart* __restrict__ ps, double gnorm, double eps_c,
               double L0, double L1, double L2, const CollBins* __restrict__ cbp,
               const int32_t* __restrict__ offs, double* __restrict__ Fc)
{
    const int w = blockIdx.x * CW_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= np)
        return;
    const CollBins cb = *cbp;
    const double h = g.h, inv_h = 1.0 / g.h, gfac = gnorm / eps_c;
    const double L[3] = {L0, L1, L2};
    const CollPart me = ps[w];
    const double xi[3] = {me.x, me.y, me.z};
    int bi[3];
    coll_bin(g, cb, xi, bi);
    int lo[3], cnt_a[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (cb.nb[a] == 1) {
            lo[a] = 0;
            cnt_a[a] = 1;
        } else if (cb.nb[a] == 2 && g.periodic[a]) {
            lo[a] = 0;
            cnt_a[a] = 2;
        } else {
            lo[a] = -1;
            cnt_a[a] = 3;
        }
    }
    const int nv = cnt_a[0] * cnt_a[1] * cnt_a[2];
    int q0 = 0, cnt = 0;
    if (lane < nv) {
        const int o[3] = {lo[0] + lane % cnt_a[0], lo[1] + (lane / cnt_a[0]) % cnt_a[1],
                          lo[2] + lane / (cnt_a[0] * cnt_a[1])};
        int nbin[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int v = bi[a] + o[a];
            if (g.periodic[a])
                v = wrapi(v, cb.nb[a]);
            else if (v < 0 || v >= cb.nb[a])
                ok = false;
            nbin[a] = v;
        }
        if (ok) {
            const int bin = nbin[0] + cb.nb[0] * (nbin[1] + cb.nb[1] * nbin[2]);
            q0 = offs[bin];
            cnt = offs[bin + 1] - q0;
        }
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o)
            incl += t;
    }
    const int excl = incl - cnt;
    const int total = __shfl(incl, 63);
    double f[3] = {0.0, 0.0, 0.0};
    for (int base = 0; base < total; base += 64) {  // the same trip count on every lane
        const int v = base + lane;
        // bin of entry v: the last of the first nv lanes whose range starts at or before v
        int b = 0;
#pragma unroll
        for (int step = 16; step > 0; step >>= 1) {
            const int c = b + step;
            const int e = __shfl(excl, c < nv ? c : 0);
            if (c < nv && e <= v)
                b = c;
        }
        const int qb = __shfl(q0, b), eb = __shfl(excl, b);
        const int e = qb + v - eb;
        if (v >= total || e == w)
            continue;
        const CollPart pj = ps[e];
        double del[3] = {pj.x - xi[0], pj.y - xi[1], pj.z - xi[2]};
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (L[c] > 0.0 && !(fabs(del[c]) < 0.25 * L[c]))
                del[c] -= L[c] * floor(del[c] / L[c] + 0.5);
        const double r2 = del[0] * del[0] + del[1] * del[1] + del[2] * del[2];
        const double Dc = 0.5 * (me.d + pj.d) + h;
        if (!(r2 < Dc * Dc) || r2 == 0.0)
            continue;
        const double dist = sqrt(r2);
        if (!(dist < Dc))
            continue;
        const double qd = (dist - Dc) * inv_h;
        const double sc = 0.5 * (me.m + pj.m) * gfac * qd * qd / dist;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            f[c] -= sc * del[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            f[c] += __shfl_xor(f[c], o);
    if (lane == 0)
        for (int c = 0; c < 3; ++c)
            Fc[3 * me.id + c] = f[c];
}

// Upper bound of the bin count: at most one bin per tile and CB_MAX_BINS.
static int64_t coll_bins_max(const Grid& g)
{
    return g.ntiles < CB_MAX_BINS ? g.ntiles : CB_MAX_BINS;
}

// Workspace of the neighbour search: bin keys and sorted ids (and their sort
// scratch), bin offsets, the bin geometry, the particles in bin order.
struct CollWs {
    int32_t *keys, *vals, *tk, *tv, *offs;
    void* rs;
    CollBins* cb;
    CollPart* ps;
};

static CollWs carve_coll(const Grid& g, int32_t np, void* ws, size_t bytes, size_t* need)
{
    Carver cv(ws, bytes);
    CollWs w;
    w.keys = cv.take<int32_t>(np);
    w.vals = cv.take<int32_t>(np);
    w.tk = cv.take<int32_t>(np);
    w.tv = cv.take<int32_t>(np);
    w.offs = cv.take<int32_t>((size_t)coll_bins_max(g) + 1);
    w.rs = cv.take<char>(radix_workspace(np));
    w.cb = cv.take<CollBins>(1);
    w.ps = cv.take<CollPart>(np);
    *need = cv.used;
    return w;
}

}  // namespace ibx

using namespace ibx;

extern "C" size_t ib_collision_workspace(const ib_level* lv, int32_t np)
{
    if (check_level(lv) || np < 0)
        return 0;
    size_t need = 0;
    carve_coll(make_grid(lv), np, nullptr, 0, &need);
    return need;
}

extern "C" int ib_collision_forces(const ib_level* lv, const ib_particles* p, const double* rho_p,
                                   double g_norm, double eps_c, double* Fc, void* ws,
                                   size_t ws_bytes, void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!p || p->np < 0 || !(eps_c > 0.0) || !(g_norm >= 0.0))
        return IB_EINVAL;
    if (p->np == 0)
        return IB_OK;
    if (!p->xc || !p->d || !rho_p || !Fc)
        return IB_EINVAL;
    const Grid g = make_grid(lv);
    size_t need = 0;
    carve_coll(g, p->np, nullptr, 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    CollWs w = carve_coll(g, p->np, ws, ws_bytes, &need);
    hipStream_t st = (hipStream_t)stream;
    double L[3];
    for (int a = 0; a < 3; ++a)
        L[a] = lv->periodic[a] ? lv->n[a] * lv->h : 0.0;
    if (p->np <= CS_MAX_NP) {
        k_coll_rank<<<(unsigned)((p->np + 63) / 64), CR_THREADS, 0, st>>>(
            p->np, g, p->xc, p->d, rho_p, w.cb, w.ps, w.offs);
    } else {
        const int64_t T = coll_bins_max(g);
        k_coll_bins<<<1, CB_THREADS, 0, st>>>(p->np, p->d, lv->h, lv->n[0], lv->n[1], lv->n[2],
                                              w.cb);
        k_coll_keys<<<(unsigned)((p->np + 255) / 256), 256, 0, st>>>(p->np, g, p->xc, w.cb,
                                                                      w.keys, w.vals);
        int bits = 1;
        while (((int64_t)1 << bits) < T)
            ++bits;
        radix_sort_pairs(w.keys, w.vals, w.tk, w.tv, p->np, nullptr, bits, w.rs, st);
        lower_bounds(w.keys, p->np, nullptr, w.offs, T, st);
        k_coll_gather<<<(unsigned)((p->np + 255) / 256), 256, 0, st>>>(p->np, w.vals, p->xc, p->d,
                                                                        rho_p, w.ps);
    }
    k_collide_bins<<<(unsigned)((p->np + CW_WAVES - 1) / CW_WAVES), 64 * CW_WAVES, 0, st>>>(
        p->np, g, w.ps, g_norm, eps_c, L[0], L[1], L[2], w.cb, w.offs, Fc);
    return launch_status();
}

extern "C" int ib_rigid_update(const ib_particles* p, const double* rho_p, const double* sums_n,
                               const double* sums_np1, const double* Fc, const double* Tc,
                               const int32_t* prescribed, double rho_f, const double* grav,
                               double dt, double* up_new, double* om_new, double* xc_new,
                               void* stream)
{
    if (!p || p->np < 0 || !grav || !(dt > 0.0) || !(rho_f >= 0.0))
        return IB_EINVAL;
    if (p->np == 0)
        return IB_OK;
    if (!p->xc || !p->d || !p->up || !p->om || !rho_p || !sums_n || !sums_np1 || !up_new ||
        !om_new || !xc_new)
        return IB_EINVAL;
    k_rigid_update<<<(unsigned)((p->np + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        p->np, p->xc, p->d, p->up, p->om, rho_p, sums_n, sums_np1, Fc, Tc, prescribed, rho_f,
        grav[0], grav[1], grav[2], dt, up_new, om_new, xc_new);
    return launch_status();
}

extern "C" int ib_advect_markers(const ib_markers* m, const double* xc_n, const double* xc_np1,
                                 const double* om_n, const double* om_np1, double dt,
                                 double* x_new, double* y_new, double* z_new, void* stream)
{
    if (!m || m->nl < 0 || !(dt >= 0.0))
        return IB_EINVAL;
    if (m->nl == 0)
        return IB_OK;
    if (!m->x || !m->y || !m->z || !m->pid || !xc_n || !xc_np1 || !om_n || !om_np1 || !x_new ||
        !y_new || !z_new)
        return IB_EINVAL;
    k_advect_markers<<<(unsigned)((m->nl + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        m->nl, m->x, m->y, m->z, m->pid, xc_n, xc_np1, om_n, om_np1, dt, x_new, y_new, z_new);
    return launch_status();
}
