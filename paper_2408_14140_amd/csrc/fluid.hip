// fluid.hip -- single-level periodic fluid steps around the IB loop (Sec. 3.1):
// Step 1, the semi-implicit predictor of Eq. (31), and Step 3, the nodal
// projection of Eqs. (ns_lp1)-(ns_lp3).
//
// Grid: n^3 cells of edge h, periodic on every axis, n a power of two.
// Velocity is cell-centred [3][n][n][n] (x fastest); pressure lives on the
// nodes [n][n][n], node (i, j, k) at the low corner of cell (i, j, k).
//   G p (cell gradient of nodal p): the difference across the cell along the
//       axis, averaged over the cell's four edges parallel to it;
//   D V (nodal divergence of cell V): the difference between the two layers
//       of cells that share the node, each averaged over its four cells
//       (D = -G^T);
//   L: the 7-point Laplacian; the convective term in central flux form with
//       face values the mean of the two cells (the paper cites a Godunov
//       scheme without giving it).
// Both implicit solves are diagonal in Fourier space: a complex radix-2
// Stockham FFT along each axis (one workgroup per line, the line in LDS), a
// per-mode scaling, and the inverse.
#include "paths.h"

namespace ibx {

template <typename T>
struct Cx {
    T x, y;
};

// ------------------------------------------------------------------ FFT

// W[q] = exp(-2 pi i q / n), q < n/2.
template <typename T>
__global__ void k_twiddles(int n, Cx<T>* W)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n / 2)
        return;
    double s, c;
    sincospi(-2.0 * (double)q / (double)n, &s, &c);
    W[q].x = (T)c;
    W[q].y = (T)s;
}

// One line per workgroup (n/2 threads, one butterfly each per stage).  Line
// L along `axis`: element j at base(L) + j * stride.  INV uses the conjugate
// twiddles; every output is multiplied by `scale`.
template <typename T, bool INV>
__global__ void __launch_bounds__(512)
k_fft_lines(Cx<T>* __restrict__ data, int n, int logn, int axis, const Cx<T>* __restrict__ W,
            T scale)
{
    extern __shared__ unsigned char smem[];
    Cx<T>* a = reinterpret_cast<Cx<T>*>(smem);
    Cx<T>* b = a + n;
    Cx<T>* w = b + n;
    const int t = threadIdx.x;
    const int64_t L = blockIdx.x;
    const int64_t nn = (int64_t)n * n;
    int64_t base, stride;
    if (axis == 0) {
        base = L * n;
        stride = 1;
    } else if (axis == 1) {
        base = (L % n) + (L / n) * nn;
        stride = n;
    } else {
        base = L;
        stride = nn;
    }
    const int half = n >> 1;
    for (int j = t; j < n; j += blockDim.x)
        a[j] = data[base + j * stride];
    for (int q = t; q < half; q += blockDim.x)
        w[q] = W[q];
    __syncthreads();
    Cx<T>* src = a;
    Cx<T>* dst = b;
    for (int s = 0; s < logn; ++s) {
        const int ns = 1 << s;                     // length of the transforms done so far
        for (int i = t; i < half; i += blockDim.x) {
            const int k = i & (ns - 1), jb = i >> s;
            const Cx<T> u = src[i], v = src[i + half];
            Cx<T> tw = w[k << (logn - 1 - s)];
            if (INV)
                tw.y = -tw.y;
            Cx<T> vt;
            vt.x = tw.x * v.x - tw.y * v.y;
            vt.y = tw.x * v.y + tw.y * v.x;
            const int o = (jb << (s + 1)) + k;
            dst[o].x = u.x + vt.x;
            dst[o].y = u.y + vt.y;
            dst[o + ns].x = u.x - vt.x;
            dst[o + ns].y = u.y - vt.y;
        }
        __syncthreads();
        Cx<T>* tmp = src;
        src = dst;
        dst = tmp;
    }
    for (int j = t; j < n; j += blockDim.x) {
        Cx<T> v = src[j];
        v.x *= scale;
        v.y *= scale;
        data[base + j * stride] = v;
    }
}

// Lines along y or z, 2^lx of them side by side (consecutive x) per
// workgroup, so that every load and store moves 2^lx consecutive elements:
// LDS holds [n][2^lx] (element j of line xi at j * 2^lx + xi).
template <typename T, bool INV>
__global__ void __launch_bounds__(256)
k_fft_cols(Cx<T>* __restrict__ data, int n, int logn, int lx, int axis,
           const Cx<T>* __restrict__ W, T scale)
{
    extern __shared__ unsigned char smem[];
    const int X = 1 << lx;
    Cx<T>* a = reinterpret_cast<Cx<T>*>(smem);
    Cx<T>* b = a + (size_t)n * X;
    Cx<T>* w = b + (size_t)n * X;
    const int t = threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    const int groups_x = n >> lx;
    const int64_t x0 = (int64_t)(blockIdx.x % groups_x) << lx;
    const int64_t other = blockIdx.x / groups_x;
    const int64_t stride = axis == 1 ? n : nn;
    const int64_t base = x0 + (axis == 1 ? other * nn : other * n);
    const int half = n >> 1;
    const int tot = n << lx;
    for (int idx = t; idx < tot; idx += blockDim.x) {
        const int j = idx >> lx, xi = idx & (X - 1);
        a[idx] = data[base + xi + j * stride];
    }
    for (int q = t; q < half; q += blockDim.x)
        w[q] = W[q];
    __syncthreads();
    Cx<T>* src = a;
    Cx<T>* dst = b;
    for (int s = 0; s < logn; ++s) {
        const int ns = 1 << s;
        for (int idx = t; idx < (half << lx); idx += blockDim.x) {
            const int i = idx >> lx, xi = idx & (X - 1);
            const int k = i & (ns - 1), jb = i >> s;
            const Cx<T> u = src[(i << lx) + xi], v = src[((i + half) << lx) + xi];
            Cx<T> tw = w[k << (logn - 1 - s)];
            if (INV)
                tw.y = -tw.y;
            Cx<T> vt;
            vt.x = tw.x * v.x - tw.y * v.y;
            vt.y = tw.x * v.y + tw.y * v.x;
            const int o = (jb << (s + 1)) + k;
            dst[(o << lx) + xi].x = u.x + vt.x;
            dst[(o << lx) + xi].y = u.y + vt.y;
            dst[((o + ns) << lx) + xi].x = u.x - vt.x;
            dst[((o + ns) << lx) + xi].y = u.y - vt.y;
        }
        __syncthreads();
        Cx<T>* tmp = src;
        src = dst;
        dst = tmp;
    }
    for (int idx = t; idx < tot; idx += blockDim.x) {
        const int j = idx >> lx, xi = idx & (X - 1);
        Cx<T> v = src[idx];
        v.x *= scale;
        v.y *= scale;
        data[base + xi + j * stride] = v;
    }
}

template <typename T>
static void fft3(Cx<T>* data, int n, int logn, const Cx<T>* W, bool inv, hipStream_t st)
{
    const unsigned lines = (unsigned)((int64_t)n * n);
    const int threads = n / 2 < 64 ? 64 : (n / 2 > 512 ? 512 : n / 2);
    const size_t lds = sizeof(Cx<T>) * (2 * (size_t)n + n / 2);
    const T scale = inv ? (T)(1.0 / (double)n) : (T)1;
    if (inv)
        k_fft_lines<T, true><<<lines, threads, lds, st>>>(data, n, logn, 0, W, scale);
    else
        k_fft_lines<T, false><<<lines, threads, lds, st>>>(data, n, logn, 0, W, scale);
    // y and z: as many side-by-side lines as keep the two LDS planes and the
    // twiddles within 64 KiB (at most 16, at most n)
    int lx = 0;
    while (lx < 4 && (2 << lx) <= n &&
           (2 * (size_t)n * (2u << lx) + n / 2) * sizeof(Cx<T>) <= 65536)
        ++lx;
    const size_t ldsc = sizeof(Cx<T>) * (2 * ((size_t)n << lx) + n / 2);
    const unsigned groups = (unsigned)(((int64_t)n * n) >> lx);
    for (int axis = 1; axis < 3; ++axis) {
        if (inv)
            k_fft_cols<T, true><<<groups, 256, ldsc, st>>>(data, n, logn, lx, axis, W, scale);
        else
            k_fft_cols<T, false><<<groups, 256, ldsc, st>>>(data, n, logn, lx, axis, W, scale);
    }
}

// ------------------------------------------------------------------ stencils

struct Idx {
    int n;
    __device__ int64_t at(int i, int j, int k) const
    {
        i &= n - 1;
        j &= n - 1;
        k &= n - 1;
        return (int64_t)i + (int64_t)n * ((int64_t)j + (int64_t)n * k);
    }
};

// component d of G p at cell (i, j, k)
template <typename T>
__device__ inline T grad_node(const T* __restrict__ p, const Idx& I, int i, int j, int k, int d,
                              T inv_h)
{
    int o[3] = {0, 0, 0};
    T lo = 0, hi = 0;
    const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            o[e1] = a;
            o[e2] = b;
            o[d] = 0;
            lo += p[I.at(i + o[0], j + o[1], k + o[2])];
            o[d] = 1;
            hi += p[I.at(i + o[0], j + o[1], k + o[2])];
        }
    return (T(0.25) * hi - T(0.25) * lo) * inv_h;
}

// the same, read from values of type T and formed in A
template <typename A, typename T>
__device__ inline A grad_node_as(const T* __restrict__ p, const Idx& I, int i, int j, int k, int d,
                                 A inv_h)
{
    int o[3] = {0, 0, 0};
    A lo = 0, hi = 0;
    const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            o[e1] = a;
            o[e2] = b;
            o[d] = 0;
            lo += (A)p[I.at(i + o[0], j + o[1], k + o[2])];
            o[d] = 1;
            hi += (A)p[I.at(i + o[0], j + o[1], k + o[2])];
        }
    return (A(0.25) * hi - A(0.25) * lo) * inv_h;
}

// rhs of Eq. (31) for every cell, paired into two complex planes
template <typename T>
__global__ void k_predict_rhs(int n, T h, T rho, T a, T dt, T g0, T g1, T g2,
                              const T* __restrict__ u, const T* __restrict__ p,
                              Cx<T>* __restrict__ r)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const T inv_h = T(1) / h, inv_h2 = inv_h * inv_h;
    const T g[3] = {g0, g1, g2};
    T uc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        uc[c] = u[c * N + q];
    T conv[3] = {0, 0, 0}, lap[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int dp[3] = {d == 0, d == 1, d == 2};
        const int64_t qp = I.at(i + dp[0], j + dp[1], k + dp[2]);
        const int64_t qm = I.at(i - dp[0], j - dp[1], k - dp[2]);
        T up[3], um[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            up[c] = u[c * N + qp];
            um[c] = u[c * N + qm];
        }
        const T fd_p = T(0.5) * (uc[d] + up[d]), fd_m = T(0.5) * (um[d] + uc[d]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T fp = fd_p * (T(0.5) * (uc[c] + up[c]));
            const T fm = fd_m * (T(0.5) * (um[c] + uc[c]));
            conv[c] += (fp - fm) * inv_h;
            lap[c] += (up[c] - T(2) * uc[c] + um[c]) * inv_h2;
        }
    }
    T rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T gp = grad_node(p, I, i, j, k, c, inv_h);
        rv[c] = uc[c] - dt * conv[c] - (dt / rho) * gp + a * lap[c] + dt * g[c];
    }
    // the solve's operator is real, so two real fields share one complex
    // transform: plane 0 holds x + i y, plane 1 holds z
    Cx<T> v0, v1;
    v0.x = rv[0];
    v0.y = rv[1];
    v1.x = rv[2];
    v1.y = T(0);
    r[q] = v0;
    r[N + q] = v1;
}

// r^[c][k] /= 1 - a lam(k) on both planes, lam the 7-point eigenvalue of mode k
template <typename T>
__global__ void k_helmholtz_scale(int n, double h, double a, Cx<T>* __restrict__ r)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const int kk[3] = {(int)(q & (n - 1)), (int)((q / n) & (n - 1)), (int)(q / ((int64_t)n * n))};
    double lam = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        lam += (2.0 * cospi(2.0 * (double)kk[d] / (double)n) - 2.0) / (h * h);
    const T f = (T)(1.0 / (1.0 - a * lam));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        Cx<T> v = r[c * N + q];
        v.x *= f;
        v.y *= f;
        r[c * N + q] = v;
    }
}

// the three velocity components back from the two planes
template <typename T>
__global__ void k_unpair(int64_t N, const Cx<T>* __restrict__ r, T* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Cx<T> v0 = r[q], v1 = r[N + q];
    out[q] = v0.x;
    out[N + q] = v0.y;
    out[2 * N + q] = v1.x;
}

template <typename T>
__global__ void k_real_part(int64_t m, const Cx<T>* __restrict__ r, T* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m)
        out[q] = r[q].x;
}

template <typename T>
__global__ void k_copy(int64_t m, const T* __restrict__ a, T* __restrict__ b)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m)
        b[q] = a[q];
}

// V = u*/dt + G p_old / rho (Eq. (ns_lp1)) for every cell
template <typename T>
__global__ void k_proj_V(int n, T h, T rho, T dt, const T* __restrict__ us,
                         const T* __restrict__ p_old, T* __restrict__ V)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const T inv_h = T(1) / h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        V[c * N + q] = us[c * N + q] / dt + grad_node(p_old, I, i, j, k, c, inv_h) / rho;
}

// D V at every node, as complex numbers
template <typename T>
__global__ void k_proj_div(int n, T h, const T* __restrict__ V, Cx<T>* __restrict__ r)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const T inv_h = T(1) / h;
    T div = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T* v = V + d * N;
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        T s[2] = {0, 0};                         // layer of cells at -1 (s[0]) and 0 (s[1]) along d
#pragma unroll
        for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    int o[3];
                    o[d] = l - 1;
                    o[e1] = -a;
                    o[e2] = -b;
                    s[l] += v[I.at(i + o[0], j + o[1], k + o[2])];
                }
        div += (T(0.25) * s[1] - T(0.25) * s[0]) * inv_h;
    }
    Cx<T> c;
    c.x = div;
    c.y = T(0);
    r[q] = c;
}

// r^[k] *= rho / sigma(k), or 0 where sigma (the symbol of D G) vanishes
template <typename T>
__global__ void k_proj_scale(int n, double h, double rho, Cx<T>* __restrict__ r)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const int kk[3] = {(int)(q & (n - 1)), (int)((q / n) & (n - 1)), (int)(q / ((int64_t)n * n))};
    double s2[3], c2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double sv = sinpi((double)kk[d] / (double)n), cv = cospi((double)kk[d] / (double)n);
        s2[d] = sv * sv;
        c2[d] = cv * cv;
    }
    const double sig = -4.0 / (h * h) *
                       (s2[0] * c2[1] * c2[2] + s2[1] * c2[0] * c2[2] + s2[2] * c2[0] * c2[1]);
    // the largest |sigma| over all modes is 4/h^2 (one component at Nyquist)
    const bool keep = fabs(sig) > 1e-10 * 4.0 / (h * h);
    const T f = keep ? (T)(rho / sig) : T(0);
    Cx<T> v = r[q];
    v.x *= f;
    v.y *= f;
    r[q] = v;
}

// The FP32 projection with one step of iterative refinement.  The FFT solve
// rounds its spectrum to FP32, and the low modes of that rounding are
// amplified by up to the condition number of D G (about n^2/pi^2).  A second
// solve of the first one's residual removes that error; the residual and the
// divergences are summed in A = FP64 from the FP32 cell values (whose own
// rounding perturbs p only as much as rounding the inputs does).
//   V = u*/dt + G p_old/rho;  p1 = rho (D G)^+ D V
//   W = V - G p1/rho;  d = rho (D G)^+ D W  (D W is the residual of p1)
//   p = p1 + d;  u^{n+1} = dt (W - G d/rho)

// D V at every node summed in A from V of type T, rounded to complex T
template <typename T, typename A>
__global__ void k_proj_div_as(int n, A h, const T* __restrict__ V, Cx<T>* __restrict__ r)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const A inv_h = A(1) / h;
    A div = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T* v = V + d * N;
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        A sl[2] = {0, 0};
#pragma unroll
        for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    int o[3];
                    o[d] = l - 1;
                    o[e1] = -a;
                    o[e2] = -b;
                    sl[l] += (A)v[I.at(i + o[0], j + o[1], k + o[2])];
                }
        div += (A(0.25) * sl[1] - A(0.25) * sl[0]) * inv_h;
    }
    Cx<T> c;
    c.x = (T)div;
    c.y = T(0);
    r[q] = c;
}

// W = V - G p/rho, in place, formed in A
template <typename T, typename A>
__global__ void k_proj_W(int n, A h, A rho, const T* __restrict__ p, T* __restrict__ V)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const A inv_h = A(1) / h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        V[c * N + q] = (T)((A)V[c * N + q] - grad_node_as<A>(p, I, i, j, k, c, inv_h) / rho);
}

// u^{n+1} = dt (W - G d/rho) and p = p1 + d
template <typename T, typename A>
__global__ void k_proj_final_refined(int n, A h, A rho, A dt, const T* __restrict__ W,
                                     const T* __restrict__ p1, const T* __restrict__ dl,
                                     T* __restrict__ un, T* __restrict__ pn)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const A inv_h = A(1) / h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        un[c * N + q] = (T)(dt * ((A)W[c * N + q] - grad_node_as<A>(dl, I, i, j, k, c, inv_h) / rho));
    pn[q] = (T)((A)p1[q] + (A)dl[q]);
}

// u^{n+1} = dt (V - G p / rho), Eq. (ns_lp3)
template <typename T>
__global__ void k_proj_final(int n, T h, T rho, T dt, const T* __restrict__ V, const T* __restrict__ pr,
                             T* __restrict__ un)
{
    const int64_t N = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N)
        return;
    const Idx I{n};
    const int i = (int)(q & (n - 1)), j = (int)((q / n) & (n - 1)), k = (int)(q / ((int64_t)n * n));
    const T inv_h = T(1) / h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        un[c * N + q] = dt * (V[c * N + q] - grad_node(pr, I, i, j, k, c, inv_h) / rho);
}

// ------------------------------------------------------------------ layouts

template <typename T>
__global__ void k_to_boxes(Grid g, const T* __restrict__ glob, T* __restrict__ boxed)
{
    const int64_t cells = (int64_t)g.box * g.box * g.box;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)g.nbox * cells)
        return;
    const int bid = (int)(q / cells);
    const int64_t r = q - (int64_t)bid * cells;
    const int lx = (int)(r % g.box), ly = (int)((r / g.box) % g.box), lz = (int)(r / ((int64_t)g.box * g.box));
    const int cx = g.box_lo[3 * bid] + lx, cy = g.box_lo[3 * bid + 1] + ly,
              cz = g.box_lo[3 * bid + 2] + lz;
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t gq = cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
    const int64_t bo = (int64_t)bid * g.bstride +
                       ((int64_t)(lz + g.ngrow) * g.ext + (ly + g.ngrow)) * g.ext + lx + g.ngrow;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        boxed[bo + c * g.cstride] = glob[c * N + gq];
}

template <typename T>
__global__ void k_from_boxes(Grid g, const T* __restrict__ boxed, T* __restrict__ glob)
{
    const int64_t cells = (int64_t)g.box * g.box * g.box;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)g.nbox * cells)
        return;
    const int bid = (int)(q / cells);
    const int64_t r = q - (int64_t)bid * cells;
    const int lx = (int)(r % g.box), ly = (int)((r / g.box) % g.box), lz = (int)(r / ((int64_t)g.box * g.box));
    const int cx = g.box_lo[3 * bid] + lx, cy = g.box_lo[3 * bid + 1] + ly,
              cz = g.box_lo[3 * bid + 2] + lz;
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t gq = cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
    const int64_t bo = (int64_t)bid * g.bstride +
                       ((int64_t)(lz + g.ngrow) * g.ext + (ly + g.ngrow)) * g.ext + lx + g.ngrow;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        glob[c * N + gq] = boxed[bo + c * g.cstride];
}

// ------------------------------------------------------------------ host

static int log2_exact(int32_t n)
{
    int l = 0;
    while ((1 << l) < n)
        ++l;
    return (1 << l) == n ? l : -1;
}

template <typename T>
struct FluidWs {
    Cx<T>* r;      // [2][N] complex
    T* V;          // [3][N]
    Cx<T>* W;      // [n/2] twiddles
};

template <typename T>
static FluidWs<T> carve_fluid(int32_t n, void* ws, size_t bytes, size_t* need)
{
    Carver cv(ws, bytes);
    const size_t N = (size_t)n * n * n;
    FluidWs<T> w;
    w.r = cv.take<Cx<T>>(2 * N);
    w.V = cv.take<T>(3 * N);
    w.W = cv.take<Cx<T>>(n / 2 > 0 ? n / 2 : 1);
    *need = cv.used;
    return w;
}

template <typename T>
static int predict_t(int32_t n, double h, double rho, double mu, double dt, const double* grav,
                     const T* u, const T* p, T* ustar, void* ws, size_t ws_bytes, hipStream_t st)
{
    size_t need = 0;
    carve_fluid<T>(n, nullptr, 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    FluidWs<T> w = carve_fluid<T>(n, ws, ws_bytes, &need);
    const int logn = log2_exact(n);
    const int64_t N = (int64_t)n * n * n;
    const unsigned gc = (unsigned)((N + 255) / 256);
    const double a = 0.5 * (mu / rho) * dt;
    k_twiddles<T><<<(unsigned)((n / 2 + 255) / 256), 256, 0, st>>>(n, w.W);
    k_predict_rhs<T><<<gc, 256, 0, st>>>(n, (T)h, (T)rho, (T)a, (T)dt, (T)grav[0], (T)grav[1],
                                         (T)grav[2], u, p, w.r);
    for (int c = 0; c < 2; ++c)
        fft3<T>(w.r + c * N, n, logn, w.W, false, st);
    k_helmholtz_scale<T><<<gc, 256, 0, st>>>(n, h, a, w.r);
    for (int c = 0; c < 2; ++c)
        fft3<T>(w.r + c * N, n, logn, w.W, true, st);
    k_unpair<T><<<gc, 256, 0, st>>>(N, w.r, ustar);
    return launch_status();
}

template <typename T>
static int project_t(int32_t n, double h, double rho, double dt, const T* ustar, const T* p_old,
                     T* u_new, T* p_new, void* ws, size_t ws_bytes, hipStream_t st)
{
    size_t need = 0;
    carve_fluid<T>(n, nullptr, 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    FluidWs<T> w = carve_fluid<T>(n, ws, ws_bytes, &need);
    const int logn = log2_exact(n);
    const int64_t N = (int64_t)n * n * n;
    const unsigned gc = (unsigned)((N + 255) / 256);
    k_twiddles<T><<<(unsigned)((n / 2 + 255) / 256), 256, 0, st>>>(n, w.W);
    if constexpr (sizeof(T) == 4) {
        // FP32: two solves, the divergences and the residual summed in FP64;
        // p1 and the correction as reals in the second complex plane
        T* p1 = reinterpret_cast<T*>(w.r + N);
        T* dl = p1 + N;
        k_proj_V<T><<<gc, 256, 0, st>>>(n, (T)h, (T)rho, (T)dt, ustar, p_old, w.V);
        k_proj_div_as<T, double><<<gc, 256, 0, st>>>(n, h, w.V, w.r);
        fft3<T>(w.r, n, logn, w.W, false, st);
        k_proj_scale<T><<<gc, 256, 0, st>>>(n, h, rho, w.r);
        fft3<T>(w.r, n, logn, w.W, true, st);
        k_real_part<T><<<gc, 256, 0, st>>>(N, w.r, p1);
        k_proj_W<T, double><<<gc, 256, 0, st>>>(n, h, rho, p1, w.V);
        k_proj_div_as<T, double><<<gc, 256, 0, st>>>(n, h, w.V, w.r);
        fft3<T>(w.r, n, logn, w.W, false, st);
        k_proj_scale<T><<<gc, 256, 0, st>>>(n, h, rho, w.r);
        fft3<T>(w.r, n, logn, w.W, true, st);
        k_real_part<T><<<gc, 256, 0, st>>>(N, w.r, dl);
        k_proj_final_refined<T, double><<<gc, 256, 0, st>>>(n, h, rho, dt, w.V, p1, dl, u_new,
                                                             p_new);
        return launch_status();
    }
    k_proj_V<T><<<gc, 256, 0, st>>>(n, (T)h, (T)rho, (T)dt, ustar, p_old, w.V);
    k_proj_div<T><<<gc, 256, 0, st>>>(n, (T)h, w.V, w.r);
    fft3<T>(w.r, n, logn, w.W, false, st);
    k_proj_scale<T><<<gc, 256, 0, st>>>(n, h, rho, w.r);
    fft3<T>(w.r, n, logn, w.W, true, st);
    // p as reals in the (unused) second complex plane, then u^{n+1}, then p_new
    T* pr = reinterpret_cast<T*>(w.r + N);
    k_real_part<T><<<gc, 256, 0, st>>>(N, w.r, pr);
    k_proj_final<T><<<gc, 256, 0, st>>>(n, (T)h, (T)rho, (T)dt, w.V, pr, u_new);
    k_copy<T><<<gc, 256, 0, st>>>(N, pr, p_new);
    return launch_status();
}

}  // namespace ibx

using namespace ibx;

static int check_fluid(int32_t n, double h, ib_prec prec)
{
    if (n < 8 || n > 1024 || log2_exact(n) < 0)
        return IB_EUNSUPPORTED;
    if (!(h > 0.0) || (prec != IB_F32 && prec != IB_F64))
        return IB_EINVAL;
    return IB_OK;
}

extern "C" size_t ib_fluid_workspace(int32_t n, ib_prec prec)
{
    if (check_fluid(n, 1.0, prec))
        return 0;
    size_t need = 0;
    if (prec == IB_F64)
        carve_fluid<double>(n, nullptr, 0, &need);
    else
        carve_fluid<float>(n, nullptr, 0, &need);
    return need;
}

extern "C" int ib_fluid_predict(int32_t n, double h, ib_prec prec, double rho, double mu,
                                double dt, const double* grav, const void* u, const void* p,
                                void* ustar, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_fluid(n, h, prec);
    if (rc)
        return rc;
    if (!(rho > 0.0) || !(mu >= 0.0) || !(dt > 0.0) || !grav || !u || !p || !ustar)
        return IB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (prec == IB_F64)
        return predict_t<double>(n, h, rho, mu, dt, grav, (const double*)u, (const double*)p,
                                 (double*)ustar, ws, ws_bytes, st);
    return predict_t<float>(n, h, rho, mu, dt, grav, (const float*)u, (const float*)p,
                            (float*)ustar, ws, ws_bytes, st);
}

extern "C" int ib_fluid_project(int32_t n, double h, ib_prec prec, double rho, double dt,
                                const void* ustar, const void* p_old, void* u_new, void* p_new,
                                void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_fluid(n, h, prec);
    if (rc)
        return rc;
    if (!(rho > 0.0) || !(dt > 0.0) || !ustar || !p_old || !u_new || !p_new)
        return IB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (prec == IB_F64)
        return project_t<double>(n, h, rho, dt, (const double*)ustar, (const double*)p_old,
                                 (double*)u_new, (double*)p_new, ws, ws_bytes, st);
    return project_t<float>(n, h, rho, dt, (const float*)ustar, (const float*)p_old,
                            (float*)u_new, (float*)p_new, ws, ws_bytes, st);
}

extern "C" int ib_field_to_boxes(const ib_level* lv, ib_prec prec, const void* glob, void* boxed,
                                 void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!glob || !boxed || (prec != IB_F32 && prec != IB_F64))
        return IB_EINVAL;
    const Grid g = make_grid(lv);
    const int64_t m = (int64_t)g.nbox * g.box * g.box * g.box;
    if (m == 0)
        return IB_OK;
    const unsigned gb = (unsigned)((m + 255) / 256);
    if (prec == IB_F64)
        k_to_boxes<double><<<gb, 256, 0, (hipStream_t)stream>>>(g, (const double*)glob,
                                                                 (double*)boxed);
    else
        k_to_boxes<float><<<gb, 256, 0, (hipStream_t)stream>>>(g, (const float*)glob,
                                                                (float*)boxed);
    return launch_status();
}

extern "C" int ib_field_from_boxes(const ib_level* lv, ib_prec prec, const void* boxed,
                                   void* glob, void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!glob || !boxed || (prec != IB_F32 && prec != IB_F64))
        return IB_EINVAL;
    const Grid g = make_grid(lv);
    const int64_t m = (int64_t)g.nbox * g.box * g.box * g.box;
    if (m == 0)
        return IB_OK;
    const unsigned gb = (unsigned)((m + 255) / 256);
    if (prec == IB_F64)
        k_from_boxes<double><<<gb, 256, 0, (hipStream_t)stream>>>(g, (const double*)boxed,
                                                                   (double*)glob);
    else
        k_from_boxes<float><<<gb, 256, 0, (hipStream_t)stream>>>(g, (const float*)boxed,
                                                                  (float*)glob);
    return launch_status();
}
