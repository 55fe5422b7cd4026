// reduce.hip -- a10: per-particle sums for the rigid-body update,
// Eqs. (particle1), (particle2) and (FD):
//   out[p][0:3]  = sum_l F_l dV_p
//   out[p][3:6]  = sum_l R_l x F_l dV_p,            R_l = X_l - X_p
//   out[p][6:9]  = sum_x alpha_p(x) u(x) h^3
//   out[p][9:12] = sum_x alpha_p(x) (x - X_p) x u(x) h^3
// alpha_p is the particle volume fraction of a cell from the eight nodal
// level-set values phi = |x_node - X_p| / (D_p/2) - 1 (Sec. 4.1, Eq.
// (level-set function)): alpha = sum over nodes with phi < 0 of -phi, divided
// by sum |phi| (0 when that sum is 0).  One workgroup per particle; every sum
// is accumulated in FP64 and combined by a fixed-shape tree, so results are
// reproducible bit for bit.
#include "paths.h"

namespace ibx {

constexpr int RD_THREADS = 1024;
constexpr int RD_WAVES = RD_THREADS / 64;

__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// One workgroup per particle.  Lanes run along x (coalesced field reads) and
// the workgroup's 32 lane groups take the y rows of the particle's bounding
// box for every z plane; wraps and box indices are formed once per column,
// plane and row rather than per cell.
template <typename T>
__global__ void __launch_bounds__(RD_THREADS)
k_particle_sums(Grid g, int32_t np, const double* __restrict__ xc, const double* __restrict__ d,
                const int64_t* __restrict__ offs, const double* __restrict__ x,
                const double* __restrict__ y, const double* __restrict__ z,
                const double* __restrict__ dv, const T* __restrict__ F,
                const T* __restrict__ u, double* __restrict__ out, int32_t* flag)
{
    __shared__ double red[RD_WAVES][12];
    const int p = blockIdx.x;
    const int t = threadIdx.x;
    const double c[3] = {xc[3 * p], xc[3 * p + 1], xc[3 * p + 2]};
    double acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q)
        acc[q] = 0.0;

    // Lagrangian sums over the particle's markers
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

    // Eulerian volume integrals over the particle's bounding cells
    const double R = 0.5 * d[p];
    const double h = g.h, h3 = h * h * h;
    int i0[3], ne[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = __ddiv_rn(__dsub_rn(c[a], g.lo[a]), h);
        const double e = R / h;
        i0[a] = (int)floor(s - e) - 1;
        ne[a] = ((int)floor(s + e) + 1) - i0[a] + 1;
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
    const int lx = t & 31, grp = t >> 5, ngrp = RD_THREADS / 32;
    // per-axis cell -> (wrapped cell, box index, index inside the box's extent)
    auto place = [&](int a, int i, int& bi, int& li) {
        int cidx = i;
        if (g.periodic[a]) {
            if (cidx < 0) cidx += g.n[a];
            else if (cidx >= g.n[a]) cidx -= g.n[a];
            if (cidx < 0 || cidx >= g.n[a]) cidx = wrapi(i, g.n[a]);
        } else if (cidx < 0 || cidx >= g.n[a]) {
            return false;
        }
        bi = cidx / g.box;
        li = cidx - bi * g.box + g.ngrow;
        return true;
    };
    int byq[2] = {0, 0}, lyq[2] = {0, 0};
    bool oky[2] = {false, false};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int jj = grp + q * ngrp;
        if (jj < ne[1])
            oky[q] = place(1, i0[1] + jj, byq[q], lyq[q]);
    }
    for (int ii = lx; g.nbox > 0 && ii < ne[0]; ii += 32) {
        const int i = i0[0] + ii;
        const double r0 = g.lo[0] + ((double)i + 0.5) * h - c[0];
        int bxi = 0, lxo = 0;
        const bool okx = place(0, i, bxi, lxo);
        for (int kk = 0; kk < ne[2]; ++kk) {
            const int k = i0[2] + kk;
            const double r2 = g.lo[2] + ((double)k + 0.5) * h - c[2];
            int bzi = 0, lzo = 0;
            const bool okz = place(2, k, bzi, lzo);
            for (int q = 0; grp + q * ngrp < ne[1]; ++q) {
                const int jj = grp + q * ngrp;
                const int j = i0[1] + jj;
                int by = 0, ly = 0;
                bool okyq;
                if (q < 2) {
                    by = byq[q];
                    ly = lyq[q];
                    okyq = oky[q];
                } else {
                    okyq = place(1, j, by, ly);
                }
                const double r1 = g.lo[1] + ((double)j + 0.5) * h - c[1];
                const double rc2 = r0 * r0 + r1 * r1 + r2 * r2;
                if (rc2 > rout2)
                    continue;
                double al = 1.0;
                if (rc2 >= rin2) {
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
                    al = den > 0.0 ? num / den : 0.0;
                    if (al == 0.0)
                        continue;
                }
                const int id = okx && okyq && okz ? g.lut[bxi + g.nb[0] * (by + g.nb[1] * bzi)]
                                                  : -1;
                if (id < 0) {
                    if (flag)
                        atomicOr(flag, 1);
                    continue;
                }
                const int64_t off = (int64_t)id * g.bstride +
                                    ((int64_t)lzo * g.ext + ly) * g.ext + lxo;
                const double u0 = (double)u[off], u1 = (double)u[off + g.cstride],
                             u2 = (double)u[off + 2 * g.cstride];
                const double wgt = al * h3;
                acc[6] += u0 * wgt;
                acc[7] += u1 * wgt;
                acc[8] += u2 * wgt;
                acc[9] += (r1 * u2 - r2 * u1) * wgt;
                acc[10] += (r2 * u0 - r0 * u2) * wgt;
                acc[11] += (r0 * u1 - r1 * u0) * wgt;
            }
        }
    }

    // fixed-shape reduction: within each wavefront, then over the wavefronts
#pragma unroll
    for (int q = 0; q < 12; ++q)
        acc[q] = wave_sum_f64(acc[q]);
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 12; ++q)
            red[t >> 6][q] = acc[q];
    }
    __syncthreads();
    if (t < 12) {
        double v = 0.0;
        for (int w = 0; w < RD_WAVES; ++w)
            v += red[w][t];
        out[12 * (int64_t)p + t] = v;
    }
}

}  // namespace ibx

using namespace ibx;

extern "C" int ib_particle_reductions(const ib_level* lv, const ib_particles* p,
                                      const ib_markers* m, ib_prec prec, const void* F,
                                      const void* u, double* out, int32_t* flag, void* stream)
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
    Grid g = make_grid(lv);
    hipStream_t st = (hipStream_t)stream;
    if (prec == IB_F64)
        k_particle_sums<double><<<(unsigned)p->np, RD_THREADS, 0, st>>>(
            g, p->np, p->xc, p->d, m->offs, m->x, m->y, m->z, m->dv, (const double*)F,
            (const double*)u, out, flag);
    else
        k_particle_sums<float><<<(unsigned)p->np, RD_THREADS, 0, st>>>(
            g, p->np, p->xc, p->d, m->offs, m->x, m->y, m->z, m->dv, (const float*)F,
            (const float*)u, out, flag);
    return launch_status();
}
