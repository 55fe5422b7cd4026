// common.hip -- host helpers shared by the libibx entry points: level checks,
// device grid descriptor, HIP error capture, status strings, and a1/a3.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "ibx_internal.h"

namespace ibx {

static thread_local char g_hip_error[256] = "";

void set_hip_error(hipError_t e)
{
    snprintf(g_hip_error, sizeof(g_hip_error), "%s: %s", hipGetErrorName(e),
             hipGetErrorString(e));
}

int launch_status()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error(e);
        return IB_EHIP;
    }
    return IB_OK;
}

int check_level(const ib_level* lv)
{
    if (!lv || !(lv->h > 0.0) || lv->box <= 0 || lv->box % TILE || lv->ngrow < 0 ||
        lv->nbox < 0 || !lv->box_lut || (lv->nbox > 0 && !lv->box_lo))
        return IB_EINVAL;
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (lv->n[a] <= 0 || lv->n[a] % lv->box)
            return IB_EINVAL;
        if (lv->periodic[a] != 0 && lv->periodic[a] != 1)
            return IB_EINVAL;
        if (!isfinite(lv->lo[a]))
            return IB_EINVAL;
        cells *= lv->n[a];
    }
    if (cells > (int64_t)INT32_MAX)
        return IB_EINVAL;
    return IB_OK;
}

Grid make_grid(const ib_level* lv)
{
    Grid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = lv->n[a];
        g.periodic[a] = lv->periodic[a];
        g.nb[a] = lv->n[a] / lv->box;
        g.nt[a] = lv->n[a] / TILE;
        g.lo[a] = lv->lo[a];
    }
    g.box = lv->box;
    g.ngrow = lv->ngrow;
    g.ext = lv->box + 2 * lv->ngrow;
    g.cstride = (int64_t)g.ext * g.ext * g.ext;
    g.bstride = 3 * g.cstride;
    g.h = lv->h;
    g.inv_h3 = 1.0 / (lv->h * lv->h * lv->h);
    g.lut = lv->box_lut;
    g.box_lo = lv->box_lo;
    g.nbox = lv->nbox;
    g.ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    return g;
}

// ------------------------------------------------------------------ a1 markers

// One workgroup per particle; marker l of N sits at height z_l = 1-(2l+1)/N
// on the unit sphere, azimuth l times the golden angle pi(3 - sqrt 5).
__global__ void k_build_markers(int32_t np, const double* __restrict__ xc,
                                const double* __restrict__ d, double h,
                                const int64_t* __restrict__ offs, double* x, double* y,
                                double* z, int32_t* pid, double* dv)
{
    const int p = blockIdx.x;
    if (p >= np)
        return;
    const int64_t o = offs[p];
    const int64_t N = offs[p + 1] - o;
    const double R = 0.5 * d[p];
    const double golden = M_PI * (3.0 - sqrt(5.0));
    const double cx = xc[3 * p], cy = xc[3 * p + 1], cz = xc[3 * p + 2];
    if (threadIdx.x == 0)
        dv[p] = M_PI * h / (3.0 * (double)N) * (3.0 * d[p] * d[p] + h * h);
    for (int64_t l = threadIdx.x; l < N; l += blockDim.x) {
        const double zl = 1.0 - (2.0 * (double)l + 1.0) / (double)N;
        const double rho = sqrt(1.0 - zl * zl);
        const double th = (double)l * golden;
        double sn, cs;
        sincos(th, &sn, &cs);
        x[o + l] = cx + R * (rho * cs);
        y[o + l] = cy + R * (rho * sn);
        z[o + l] = cz + R * zl;
        pid[o + l] = p;
    }
}

// ------------------------------------------------------------------ a3 U^d

template <typename T>
__global__ void k_desired_velocity(int64_t nl, const double* __restrict__ x,
                                   const double* __restrict__ y, const double* __restrict__ z,
                                   const int32_t* __restrict__ pid, const double* __restrict__ xc,
                                   const double* __restrict__ up, const double* __restrict__ om,
                                   T* Ud)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl)
        return;
    const int p = pid[l];
    const double R0 = x[l] - xc[3 * p], R1 = y[l] - xc[3 * p + 1], R2 = z[l] - xc[3 * p + 2];
    const double w0 = om[3 * p], w1 = om[3 * p + 1], w2 = om[3 * p + 2];
    Ud[3 * l + 0] = (T)(up[3 * p + 0] + (w1 * R2 - w2 * R1));
    Ud[3 * l + 1] = (T)(up[3 * p + 1] + (w2 * R0 - w0 * R2));
    Ud[3 * l + 2] = (T)(up[3 * p + 2] + (w0 * R1 - w1 * R0));
}

void desired_velocity(const ib_particles* p, const ib_markers* m, ib_prec prec, void* Ud,
                      hipStream_t st)
{
    if (m->nl == 0)
        return;
    const unsigned gb = (unsigned)((m->nl + 255) / 256);
    if (prec == IB_F64)
        k_desired_velocity<double><<<gb, 256, 0, st>>>(m->nl, m->x, m->y, m->z, m->pid, p->xc,
                                                       p->up, p->om, (double*)Ud);
    else
        k_desired_velocity<float><<<gb, 256, 0, st>>>(m->nl, m->x, m->y, m->z, m->pid, p->xc,
                                                      p->up, p->om, (float*)Ud);
}

// ------------------------------------------------------------------ flagged buckets

// Every output of a call made with a flagged bucket set (a stencil that leaves
// the covered boxes or a bounded axis, or an overflowing source list) is set
// to NaN, so a wrong result never looks like a valid one.  Every thread reads
// the two flag words; with both clear the kernel does nothing.
template <typename T>
__global__ void __launch_bounds__(256)
k_poison(const int32_t* __restrict__ flag, Grid g, PoisonSet ps)
{
    if ((flag[0] | flag[1]) == 0)
        return;
    const T nan = (T)__builtin_nan("");
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_box = (int64_t)g.box * g.box * g.box;
    for (int k = 0; k < 2; ++k) {
        T* fld = (T*)ps.field[k];
        if (!fld)
            continue;
        for (int64_t q = t0; q < per_box * g.nbox; q += stride) {
            const int64_t bid = q / per_box, r = q - bid * per_box;
            const int lx = (int)(r % g.box) + g.ngrow;
            const int ly = (int)((r / g.box) % g.box) + g.ngrow;
            const int lz = (int)(r / ((int64_t)g.box * g.box)) + g.ngrow;
            const int64_t off = bid * g.bstride + ((int64_t)lz * g.ext + ly) * g.ext + lx;
            fld[off] = nan;
            fld[off + g.cstride] = nan;
            fld[off + 2 * g.cstride] = nan;
        }
    }
    for (int k = 0; k < 2; ++k)
        for (int64_t q = t0; ps.vec[k] && q < ps.nvec[k]; q += stride)
            ((T*)ps.vec[k])[q] = nan;
    for (int k = 0; k < 4; ++k)
        for (int64_t q = t0; ps.dvec[k] && q < ps.ndvec[k]; q += stride)
            ps.dvec[k][q] = __builtin_nan("");
}

void poison_if_flagged(const int32_t* flag, const Grid& g, ib_prec prec, const PoisonSet& ps,
                       hipStream_t st)
{
    if (!flag)
        return;
    if (prec == IB_F64)
        k_poison<double><<<512, 256, 0, st>>>(flag, g, ps);
    else
        k_poison<float><<<512, 256, 0, st>>>(flag, g, ps);
}

}  // namespace ibx

using namespace ibx;

extern "C" int64_t ib_count_markers(int32_t np, const double* d_host, double h,
                                    int64_t* offs_host)
{
    if (np < 0 || !(h > 0.0) || !offs_host || (np > 0 && !d_host))
        return IB_EINVAL;
    offs_host[0] = 0;
    for (int32_t p = 0; p < np; ++p) {
        if (!(d_host[p] > 0.0) || !isfinite(d_host[p]))
            return IB_EINVAL;
        const double q = d_host[p] / h;
        offs_host[p + 1] = offs_host[p] + (int64_t)llround(M_PI * q * q);
    }
    return offs_host[np];
}

extern "C" int ib_build_markers(const ib_level* lv, const ib_particles* p, const ib_markers* m,
                                void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!p || !m || p->np < 0 || m->nl < 0 || !m->offs || !m->dv ||
        (p->np > 0 && (!p->xc || !p->d)) || (m->nl > 0 && (!m->x || !m->y || !m->z || !m->pid)))
        return IB_EINVAL;
    if (p->np == 0)
        return IB_OK;
    k_build_markers<<<(unsigned)p->np, 256, 0, (hipStream_t)stream>>>(
        p->np, p->xc, p->d, lv->h, m->offs, m->x, m->y, m->z, m->pid, m->dv);
    return launch_status();
}

extern "C" int ib_desired_velocity(const ib_particles* p, const ib_markers* m, ib_prec prec,
                                   void* Ud, void* stream)
{
    if (!p || !m || !Ud || (prec != IB_F32 && prec != IB_F64) || m->nl < 0 ||
        (m->nl > 0 && (!m->x || !m->y || !m->z || !m->pid || !p->xc || !p->up || !p->om)))
        return IB_EINVAL;
    desired_velocity(p, m, prec, Ud, (hipStream_t)stream);
    return launch_status();
}

extern "C" const char* ib_status_string(int status)
{
    switch (status) {
    case IB_OK: return "ok";
    case IB_EINVAL: return "invalid argument";
    case IB_EDOMAIN: return "input outside the covered grid";
    case IB_EWORKSPACE: return "workspace missing or too small";
    case IB_EHIP: return "HIP runtime error";
    case IB_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
    }
}

extern "C" const char* ib_last_hip_error(void) { return ibx::g_hip_error; }

extern "C" int ib_version(void) { return 1; }
