// rigid.hip -- the particle side of a time step (Sec. 3.2; Step 4 of
// Sec. 3.1): rigid-body update of the spheres and rigid advection of their
// markers.  One thread per particle, one thread per marker; FP64 throughout.
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

// Eq. (DKT_model): F_c,ij = -(m |g| / eps_c) ((|delta| - D_c)/h)^2 delta/|delta|
// for |delta| < D_c = R_i + R_j + h, delta = X_j - X_i by the minimum image on
// periodic axes, m the mean of the two masses.  One wavefront per particle
// i: lane k takes the partners j = k, k + 64, ... in order, and the lanes'
// sums are combined by a fixed butterfly, so the result is reproducible.
constexpr int CL_WAVES = 4;

__global__ void __launch_bounds__(64 * CL_WAVES)
k_collision_forces(int32_t np, const double* __restrict__ xc, const double* __restrict__ d,
                   const double* __restrict__ rho_p, double gnorm, double h, double eps_c,
                   double L0, double L1, double L2, double* __restrict__ Fc)
{
    const int i = blockIdx.x * CL_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= np)
        return;
    const double L[3] = {L0, L1, L2};
    const double xi[3] = {xc[3 * i], xc[3 * i + 1], xc[3 * i + 2]};
    const double di = d[i];
    const double mi = rho_p[i] * 3.14159265358979323846 * di * di * di / 6.0;
    double f[3] = {0.0, 0.0, 0.0};
    for (int j = lane; j < np; j += 64) {
        if (j == i)
            continue;
        double del[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            del[c] = xc[3 * j + c] - xi[c];
            if (L[c] > 0.0)
                del[c] -= L[c] * floor(del[c] / L[c] + 0.5);
        }
        const double r2 = del[0] * del[0] + del[1] * del[1] + del[2] * del[2];
        const double dj = d[j];
        const double Dc = 0.5 * (di + dj) + h;
        if (!(r2 < Dc * Dc) || r2 == 0.0)
            continue;
        const double dist = sqrt(r2);
        if (!(dist < Dc))
            continue;
        const double mj = rho_p[j] * 3.14159265358979323846 * dj * dj * dj / 6.0;
        const double q = (dist - Dc) / h;
        const double mag = 0.5 * (mi + mj) * gnorm / eps_c * q * q;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            f[c] -= mag * del[c] / dist;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            f[c] += __shfl_xor(f[c], o);
    if (lane == 0)
        for (int c = 0; c < 3; ++c)
            Fc[3 * i + c] = f[c];
}

}  // namespace ibx

using namespace ibx;

extern "C" int ib_collision_forces(const ib_level* lv, const ib_particles* p, const double* rho_p,
                                   double g_norm, double eps_c, double* Fc, void* stream)
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
    double L[3];
    for (int a = 0; a < 3; ++a)
        L[a] = lv->periodic[a] ? lv->n[a] * lv->h : 0.0;
    k_collision_forces<<<(unsigned)((p->np + CL_WAVES - 1) / CL_WAVES), 64 * CL_WAVES, 0,
                         (hipStream_t)stream>>>(p->np, p->xc, p->d, rho_p, g_norm, lv->h, eps_c,
                                                L[0], L[1], L[2], Fc);
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
