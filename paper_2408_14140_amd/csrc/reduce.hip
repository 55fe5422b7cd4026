// reduce.hip -- a10: per-particle sums for the rigid-body update,
// Eqs. (particle1), (particle2) and (FD):
//   out[p][0:3]  = sum_l F_l dV_p
//   out[p][3:6]  = sum_l R_l x F_l dV_p,            R_l = X_l - X_p
//   out[p][6:9]  = sum_x alpha_p(x) u(x) h^3
//   out[p][9:12] = sum_x alpha_p(x) (x - X_p) x u(x) h^3
// alpha_p is the particle volume fraction of a cell from the eight nodal
// level-set values phi = |x_node - X_p| / (D_p/2) - 1 (Sec. 4.1, Eq.
// (level-set function)): alpha = sum over nodes with phi < 0 of -phi, divided
// by sum |phi| (0 when that sum is 0).
//
// The volume integrals run on RD_SLABS workgroups per particle, each taking
// the z planes of the particle's bounding box congruent to its slab index,
// and write FP64 partial sums; one more workgroup per particle forms the
// Lagrangian sums beside them, and a second kernel adds the slab partials in
// a fixed order.  Every sum is formed by fixed-shape
// trees, so results are reproducible bit for bit.
#include <mutex>

#include "paths.h"

namespace ibx {

constexpr int RD_THREADS = 256;
constexpr int RD_WAVES = RD_THREADS / 64;
constexpr int RD_SLABS = 4;
constexpr int RD_QCAP = 512;               // per-wavefront queue capacity (cells)
constexpr int RD_TAB = 256;                // bounding-box cells per axis held in LDS tables

__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// Fixed-shape sum of n values over a workgroup of RD_THREADS: wavefronts
// first, then the wavefront sums in order.  Result valid in thread 0.
template <int N>
__device__ inline void block_sums(double (&acc)[N], double (*red)[N])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < N; ++q)
        acc[q] = wave_sum_f64(acc[q]);
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q)
            red[t >> 6][q] = acc[q];
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double v = 0.0;
            for (int w = 0; w < RD_WAVES; ++w)
                v += red[w][q];
            acc[q] = v;
        }
    }
}

// Lagrangian sums of particle p -> part[p][RD_SLABS][6].
template <typename T>
__device__ void lagrangian_sums(int p, const double* __restrict__ xc,
                                const int64_t* __restrict__ offs, const double* __restrict__ x,
                                const double* __restrict__ y, const double* __restrict__ z,
                                const double* __restrict__ dv, const T* __restrict__ F,
                                double* __restrict__ part, double (*red)[6])
{
    const int t = threadIdx.x;
    const double c[3] = {xc[3 * p], xc[3 * p + 1], xc[3 * p + 2]};
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double dvp = dv[p];
    for (int64_t l = offs[p] + t; l < offs[p + 1]; l += RD_THREADS) {
        const double F0 = (double)F[3 * l], F1 = (double)F[3 * l + 1], F2 = (double)F[3 * l + 2];
        const double R0 = x[l] - c[0], R1 = y[l] - c[1], R2 = z[l] - c[2];
        acc[0] += F0 * dvp;
        acc[1] += F1 * dvp;
        acc[2] += F2 * dvp;
        acc[3] += (R1 * F2 - R2 * F1) * dvp;
        acc[4] += (R2 * F0 - R0 * F2) * dvp;
        acc[5] += (R0 * F1 - R1 * F0) * dvp;
    }
    block_sums<6>(acc, red);
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            part[((int64_t)p * (RD_SLABS + 1) + RD_SLABS) * 6 + q] = acc[q];
    }
}

// Volume integrals of particle blockIdx.x over the z planes kk = slab,
// slab + RD_SLABS, ... of its bounding box -> part[p][slab][6]; workgroup
// slab = RD_SLABS forms the particle's Lagrangian sums instead.
// Each wavefront classifies 64 cells per round with no global access:
// interior cells (alpha = 1) and cells near the surface go, in cell order, to
// two queues of its own in LDS, drained in bulk with independent loads.
template <typename T>
__global__ void __launch_bounds__(RD_THREADS)
k_volume_partials(Grid g, const double* __restrict__ xc, const double* __restrict__ d,
                  const T* __restrict__ u, double* __restrict__ part, int32_t* flag,
                  const int64_t* __restrict__ offs, const double* __restrict__ mx,
                  const double* __restrict__ my, const double* __restrict__ mz,
                  const double* __restrict__ dv, const T* __restrict__ F)
{
    __shared__ double red[RD_WAVES][6];
    __shared__ int qin[RD_WAVES * RD_QCAP], qsurf[RD_WAVES * RD_QCAP];
    __shared__ int2 ptab[3][RD_TAB];       // per axis: (box index or -1, index in the extent)
    const int p = blockIdx.x, slab = blockIdx.y;
    if (slab == RD_SLABS) {
        lagrangian_sums<T>(p, xc, offs, mx, my, mz, dv, F, part, red);
        return;
    }
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const double c[3] = {xc[3 * p], xc[3 * p + 1], xc[3 * p + 2]};
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double R = 0.5 * d[p];
    const double h = g.h, h3 = h * h * h;
    // Only a cell with a node inside the sphere has alpha != 0, and such a
    // node n satisfies |n - s| < e along every axis (s = centre, e = R, in
    // cells), so the cells floor(s - e) .. floor(s + e) hold all of them; the
    // 1e-6 cell margin is far above the rounding of s, e and phi.
    int i0[3], ne[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = __ddiv_rn(__dsub_rn(c[a], g.lo[a]), h);
        const double e = R / h;
        i0[a] = (int)floor(s - e - 1e-6);
        ne[a] = (int)floor(s + e + 1e-6) - i0[a] + 1;
    }
    const double invR = 1.0 / R;
    // A cell whose centre lies farther than half its diagonal (plus a margin
    // far above rounding) inside the sphere has all eight nodal phi < 0, so
    // the formula gives exactly 1 (its numerator and denominator add the same
    // terms); one as far outside has all phi > 0 and gives exactly 0.  Only
    // the cells near the surface evaluate the eight nodes.
    const double hc = 0.8660254037844386 * h, margin = 1e-9 * R;
    const double rin = R - hc - margin, rout = R + hc + margin;
    const double rin2 = rin > 0.0 ? rin * rin : -1.0, rout2 = rout * rout;
    // floor(a / b) for 0 <= a < 2^31 and b < 2^20 from a double reciprocal:
    // the product's error (a few units in 2^-52 relative) stays far below the
    // bias, and the bias below the 1/b gap to the next integer
    auto qdiv = [](int a, double rb) { return (int)((double)a * rb + 1e-6); };
    const double r_ne0 = 1.0 / ne[0], r_box = 1.0 / g.box;
    // this slab's cells: planes kk = slab + RD_SLABS * m
    const int nplanes = ne[2] > slab ? (ne[2] - slab + RD_SLABS - 1) / RD_SLABS : 0;
    const int plane = ne[0] * ne[1];
    const int ncell = nplanes * plane;
    const double r_plane = 1.0 / plane;
    auto decode = [&](int q, int& i, int& j, int& k) {
        const int m = qdiv(q, r_plane);
        const int rem = q - m * plane;
        const int row = qdiv(rem, r_ne0);
        i = i0[0] + (rem - row * ne[0]);
        j = i0[1] + row;
        k = i0[2] + slab + RD_SLABS * m;
    };
    auto place = [&](int a, int i, int& bi, int& li) {
        int cidx = i;
        if (g.periodic[a]) {
            if (cidx < 0) cidx += g.n[a];
            else if (cidx >= g.n[a]) cidx -= g.n[a];
            if (cidx < 0 || cidx >= g.n[a]) cidx = wrapi(i, g.n[a]);
        } else if (cidx < 0 || cidx >= g.n[a]) {
            return false;
        }
        bi = qdiv(cidx, r_box);
        li = cidx - bi * g.box + g.ngrow;
        return true;
    };
    auto alpha = [&](int i, int j, int k) {
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int dk = 0; dk < 2; ++dk)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int di = 0; di < 2; ++di) {
                    const double ex = (g.lo[0] + (double)(i + di) * h - c[0]) * invR;
                    const double ey = (g.lo[1] + (double)(j + dj) * h - c[1]) * invR;
                    const double ez = (g.lo[2] + (double)(k + dk) * h - c[2]) * invR;
                    const double phi = sqrt(ex * ex + ey * ey + ez * ez) - 1.0;
                    if (phi < 0.0)
                        num -= phi;
                    den += fabs(phi);
                }
        return den > 0.0 ? num / den : 0.0;
    };
    // placement of the bounding box's cells along each axis, formed once
    const bool tabled = ne[0] <= RD_TAB && ne[1] <= RD_TAB && nplanes <= RD_TAB;
    if (tabled) {
        for (int e = t; e < ne[0] + ne[1] + nplanes; e += RD_THREADS) {
            const int a = e < ne[0] ? 0 : e < ne[0] + ne[1] ? 1 : 2;
            const int idx = a == 0 ? e : a == 1 ? e - ne[0] : e - ne[0] - ne[1];
            const int cell = a == 2 ? i0[2] + slab + RD_SLABS * idx : i0[a] + idx;
            int bi = -1, li = 0;
            if (!place(a, cell, bi, li))
                bi = -1;
            ptab[a][idx] = make_int2(bi, li);
        }
    }
    __syncthreads();
    auto add_cell = [&](int i, int j, int k, double al) {
        int bx = -1, lxo = 0, by = -1, lyo = 0, bz = -1, lzo = 0;
        if (tabled) {
            const int2 px = ptab[0][i - i0[0]], py = ptab[1][j - i0[1]],
                       pz = ptab[2][(k - i0[2] - slab) / RD_SLABS];
            bx = px.x; lxo = px.y; by = py.x; lyo = py.y; bz = pz.x; lzo = pz.y;
        } else if (!(place(0, i, bx, lxo) && place(1, j, by, lyo) && place(2, k, bz, lzo))) {
            bx = -1;
        }
        const bool ok = bx >= 0 && by >= 0 && bz >= 0;
        const int id = ok ? g.lut[bx + g.nb[0] * (by + g.nb[1] * bz)] : -1;
        if (id < 0) {
            if (flag)
                atomicOr(flag, 1);
            for (int q = 0; q < 6; ++q)
                acc[q] = __builtin_nan("");
            return;
        }
        const int64_t off = (int64_t)id * g.bstride + ((int64_t)lzo * g.ext + lyo) * g.ext + lxo;
        const double u0 = (double)u[off], u1 = (double)u[off + g.cstride],
                     u2 = (double)u[off + 2 * g.cstride];
        const double r0 = g.lo[0] + ((double)i + 0.5) * h - c[0];
        const double r1 = g.lo[1] + ((double)j + 0.5) * h - c[1];
        const double r2 = g.lo[2] + ((double)k + 0.5) * h - c[2];
        const double wgt = al * h3;
        acc[0] += u0 * wgt;
        acc[1] += u1 * wgt;
        acc[2] += u2 * wgt;
        acc[3] += (r1 * u2 - r2 * u1) * wgt;
        acc[4] += (r2 * u0 - r0 * u2) * wgt;
        acc[5] += (r0 * u1 - r1 * u0) * wgt;
    };
    // each wavefront queues and drains its own cells: no workgroup barrier
    int* const qi = qin + wv * RD_QCAP;
    int* const qs = qsurf + wv * RD_QCAP;
    int nin = 0, nsurf = 0;
    for (int base = wv * 64; g.nbox > 0 && base < ncell; base += RD_THREADS) {
        const int q = base + lane;
        int cls = 0;                       // 0 outside, 1 interior, 2 near the surface
        if (q < ncell) {
            int i, j, k;
            decode(q, i, j, k);
            const double r0 = g.lo[0] + ((double)i + 0.5) * h - c[0];
            const double r1 = g.lo[1] + ((double)j + 0.5) * h - c[1];
            const double r2 = g.lo[2] + ((double)k + 0.5) * h - c[2];
            const double rc2 = r0 * r0 + r1 * r1 + r2 * r2;
            cls = rc2 > rout2 ? 0 : rc2 < rin2 ? 1 : 2;
        }
        const uint64_t b1 = __ballot(cls == 1), b2 = __ballot(cls == 2);
        if (cls == 1)
            qi[nin + __builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0u))] = q;
        if (cls == 2)
            qs[nsurf + __builtin_amdgcn_mbcnt_hi((uint32_t)(b2 >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)b2, 0u))] = q;
        nin += __popcll(b1);
        nsurf += __popcll(b2);
        const bool last = base + RD_THREADS >= ncell;
        if (nin > RD_QCAP - 64 || last) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll 4
            for (int e = lane; e < nin; e += 64) {
                int i, j, k;
                decode(qi[e], i, j, k);
                add_cell(i, j, k, 1.0);
            }
            nin = 0;
            __builtin_amdgcn_wave_barrier();
        }
        if (nsurf > RD_QCAP - 64 || last) {
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < nsurf; e += 64) {
                int i, j, k;
                decode(qs[e], i, j, k);
                const double al = alpha(i, j, k);
                if (al != 0.0)
                    add_cell(i, j, k, al);
            }
            nsurf = 0;
            __builtin_amdgcn_wave_barrier();
        }
    }
    block_sums<6>(acc, red);
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            part[((int64_t)p * (RD_SLABS + 1) + slab) * 6 + q] = acc[q];
    }
}

// out[p] = (Lagrangian sums, then the slab partials of the volume integrals
// added in slab order); one thread per output value.
__global__ void k_particle_out(int64_t np, const double* __restrict__ part,
                               double* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 12 * np)
        return;
    const int64_t p = e / 12;
    const int q = (int)(e - 12 * p);
    const double* pp = part + p * (RD_SLABS + 1) * 6;
    double v;
    if (q < 6) {
        v = pp[RD_SLABS * 6 + q];
        // a particle whose cells leave the covered boxes gets NaN in all 12
        bool bad = false;
        for (int sl = 0; sl < RD_SLABS; ++sl)
            bad |= isnan(pp[sl * 6]);
        if (bad)
            v = __builtin_nan("");
    } else {
        v = 0.0;
        for (int sl = 0; sl < RD_SLABS; ++sl)
            v += pp[sl * 6 + (q - 6)];
    }
    out[e] = v;
}

}  // namespace ibx

using namespace ibx;

// Scratch of ib_particle_reductions_noalloc: the slab partial sums of up to
// RD_NOALLOC_MAX_NP particles (30 doubles each, 7.5 MiB), a file-scope device
// array that every device the library runs on holds until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address); it passes the address that
// hipGetSymbolAddress returned for the current device.
constexpr int32_t RD_NOALLOC_MAX_NP = IB_REDUCTIONS_NOALLOC_MAX_NP;
static __device__ __align__(256) double scratch[(size_t)RD_NOALLOC_MAX_NP * (RD_SLABS + 1) * 6];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e);
        return IB_EHIP;
    }
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return IB_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_hip_error(e);
            return IB_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return IB_OK;
}

int check_reductions(const ib_level* lv, const ib_particles* p, const ib_markers* m,
                     ib_prec prec, const void* F, const void* u, const double* out)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!p || !m || (prec != IB_F32 && prec != IB_F64) || p->np < 0 || m->nl < 0)
        return IB_EINVAL;
    if (p->np == 0)
        return IB_OK;
    if (!p->xc || !p->d || !m->offs || !m->dv || !u || !out ||
        (m->nl > 0 && (!F || !m->x || !m->y || !m->z)))
        return IB_EINVAL;
    return IB_OK;
}

// Both entry points: part holds (RD_SLABS + 1) * 6 doubles per particle, every
// one of them written by k_volume_partials before k_particle_out reads it.
int launch_reductions(const ib_level* lv, const ib_particles* p, const ib_markers* m,
                      ib_prec prec, const void* F, const void* u, double* out, int32_t* flag,
                      double* part, hipStream_t st)
{
    Grid g = make_grid(lv);
    const dim3 gv((unsigned)p->np, RD_SLABS + 1);
    if (prec == IB_F64)
        k_volume_partials<double><<<gv, RD_THREADS, 0, st>>>(
            g, p->xc, p->d, (const double*)u, part, flag, m->offs, m->x, m->y, m->z, m->dv,
            (const double*)F);
    else
        k_volume_partials<float><<<gv, RD_THREADS, 0, st>>>(
            g, p->xc, p->d, (const float*)u, part, flag, m->offs, m->x, m->y, m->z, m->dv,
            (const float*)F);
    const int64_t ne = 12 * (int64_t)p->np;
    k_particle_out<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(p->np, part, out);
    return launch_status();
}
}  // namespace

extern "C" size_t ib_reductions_workspace(int32_t np)
{
    return np > 0 ? (size_t)np * (RD_SLABS + 1) * 6 * sizeof(double) : 0;
}

extern "C" int ib_particle_reductions(const ib_level* lv, const ib_particles* p,
                                      const ib_markers* m, ib_prec prec, const void* F,
                                      const void* u, double* out, int32_t* flag, void* ws,
                                      size_t ws_bytes, void* stream)
{
    int rc = check_reductions(lv, p, m, prec, F, u, out);
    if (rc || p->np == 0)
        return rc;
    if (!ws || ws_bytes < ib_reductions_workspace(p->np))
        return IB_EWORKSPACE;
    return launch_reductions(lv, p, m, prec, F, u, out, flag, (double*)ws, (hipStream_t)stream);
}

extern "C" int ib_particle_reductions_noalloc(const ib_level* lv, const ib_particles* p,
                                              const ib_markers* m, ib_prec prec, const void* F,
                                              const void* u, double* out, int32_t* flag,
                                              void* stream)
{
    int rc = check_reductions(lv, p, m, prec, F, u, out);
    if (rc || p->np == 0)
        return rc;
    if (p->np > RD_NOALLOC_MAX_NP)
        return IB_EUNSUPPORTED;
    void* part = nullptr;
    rc = scratch_address(&part);
    if (rc)
        return rc;
    return launch_reductions(lv, p, m, prec, F, u, out, flag, (double*)part, (hipStream_t)stream);
}
