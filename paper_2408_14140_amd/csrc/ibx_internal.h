// ibx_internal.h -- device-side conventions shared by the libibx kernels.
//
// Grid: finest level of n[0] x n[1] x n[2] cells of edge h from lo, tiled into
// covered boxes of `box` cells stored as [nbox][3][E][E][E] (E = box + 2 ngrow,
// x fastest).  A cell is addressed through the box lookup table; ghost cells
// are never touched.  Tiles are 8^3 cells, numbered x fastest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ibx.h"

namespace ibx {

constexpr int TILE = 8;
constexpr int TILE_CELLS = TILE * TILE * TILE;

struct Grid {
    int32_t n[3];
    int32_t periodic[3];
    int32_t nb[3];       // boxes per axis
    int32_t nt[3];       // tiles per axis
    int32_t box, ngrow, ext;
    int64_t cstride;     // ext^3: one component of one box
    int64_t bstride;     // 3 ext^3: one box
    double h, inv_h3;
    double lo[3];
    const int32_t* lut;
    const int32_t* box_lo;
    int32_t nbox;
    int64_t ntiles;
};

// ---------------------------------------------------------------- addressing

__host__ __device__ inline int wrapi(int i, int n)
{
    int m = i % n;
    return m < 0 ? m + n : m;
}

// Grid coordinate s = (X - lo)/h, correctly rounded so that every caller
// (bucketing, weights) agrees bit for bit on floor(s).
__device__ inline double grid_coord(const Grid& g, int a, double X)
{
    return __ddiv_rn(__dsub_rn(X, g.lo[a]), g.h);
}

// Stencil base: floor(s) - 1 (3-point) or floor(s - 1/2) - 1 (4-point).
template <int P>
__device__ inline int stencil_base(double s)
{
    return P == 3 ? (int)floor(s) - 1 : (int)floor(s - 0.5) - 1;
}

// Offset of wrapped cell (cx, cy, cz) in the box layout (component 0), or -1
// when its box is not covered.
__device__ inline int64_t cell_offset(const Grid& g, int cx, int cy, int cz)
{
    int bx = cx / g.box, by = cy / g.box, bz = cz / g.box;
    int id = g.lut[bx + g.nb[0] * (by + g.nb[1] * bz)];
    if (id < 0)
        return -1;
    int lx = cx - bx * g.box + g.ngrow;
    int ly = cy - by * g.box + g.ngrow;
    int lz = cz - bz * g.box + g.ngrow;
    return (int64_t)id * g.bstride + ((int64_t)lz * g.ext + ly) * g.ext + lx;
}

// Same, for a cell given by unwrapped indices on periodic axes (bounded axes
// must already be inside the grid).
__device__ inline int64_t cell_offset_wrapped(const Grid& g, int cx, int cy, int cz)
{
    return cell_offset(g, wrapi(cx, g.n[0]), wrapi(cy, g.n[1]), wrapi(cz, g.n[2]));
}

// ---------------------------------------------------------------- kernels
// 3-point kernel of Roma, Peskin & Berger (1999), support |r| <= 3/2, and
// 4-point kernel of Peskin (2002), support |r| <= 2; both cited in Sec. 3.1.

template <typename T>
__device__ inline T kphi3(T r)
{
    T a = fabs(r);
    if (a <= T(0.5))
        return (T(1) + sqrt(T(1) - T(3) * a * a)) * T(1.0 / 3.0);
    if (a <= T(1.5)) {
        T t = T(1) - a;
        return (T(5) - T(3) * a - sqrt(T(1) - T(3) * t * t)) * T(1.0 / 6.0);
    }
    return T(0);
}

template <typename T>
__device__ inline T kphi4(T r)
{
    T a = fabs(r);
    if (a <= T(1))
        return (T(3) - T(2) * a + sqrt(T(1) + T(4) * a - T(4) * a * a)) * T(0.125);
    if (a <= T(2))
        return (T(5) - T(2) * a - sqrt(T(-7) + T(12) * a - T(4) * a * a)) * T(0.125);
    return T(0);
}

template <typename T>
__device__ inline T kdphi3(T r)
{
    T a = fabs(r), d;
    if (a <= T(0.5))
        d = -a / sqrt(T(1) - T(3) * a * a);
    else if (a <= T(1.5)) {
        T t = T(1) - a;
        d = (T(-3) - T(3) * t / sqrt(T(1) - T(3) * t * t)) * T(1.0 / 6.0);
    } else
        d = T(0);
    return r < T(0) ? -d : d;
}

template <typename T>
__device__ inline T kdphi4(T r)
{
    T a = fabs(r), d;
    if (a <= T(1))
        d = (T(-2) + (T(2) - T(4) * a) / sqrt(T(1) + T(4) * a - T(4) * a * a)) * T(0.125);
    else if (a <= T(2))
        d = (T(-2) - (T(6) - T(4) * a) / sqrt(T(-7) + T(12) * a - T(4) * a * a)) * T(0.125);
    else
        d = T(0);
    return r < T(0) ? -d : d;
}

template <typename T, int P>
__device__ inline T kphi(T r)
{
    return P == 3 ? kphi3<T>(r) : kphi4<T>(r);
}

template <typename T, int P>
__device__ inline T kdphi(T r)
{
    return P == 3 ? kdphi3<T>(r) : kdphi4<T>(r);
}

// One axis of a marker's stencil: unwrapped base and the P weights.
// r_a = s - (b + a) - 1/2 is formed in FP64, then rounded to T.
template <typename T, int P>
__device__ inline int axis_weights(double s, T* w)
{
    int b = stencil_base<P>(s);
    double r0 = s - (double)b - 0.5;
#pragma unroll
    for (int a = 0; a < P; ++a)
        w[a] = kphi<T, P>((T)(r0 - (double)a));
    return b;
}

template <typename T, int P>
__device__ inline int axis_weights_d(double s, T* w, T* dw)
{
    int b = stencil_base<P>(s);
    double r0 = s - (double)b - 0.5;
#pragma unroll
    for (int a = 0; a < P; ++a) {
        T r = (T)(r0 - (double)a);
        w[a] = kphi<T, P>(r);
        dw[a] = kdphi<T, P>(r);
    }
    return b;
}

// ---------------------------------------------------------------- scans

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Up to this many tiles, each workgroup of the add pass sums the tile totals
// before its own tile itself, instead of a second scan over the totals (two
// launches fewer; the sums grow with the square of the tile count).
constexpr int64_t SCAN_FUSE = 64;

// Sum of a[0 .. m) over the workgroup; every thread gets it.  Called by all
// threads of the workgroup.
__device__ inline int32_t group_sum(const int32_t* a, int64_t m)
{
    __shared__ int32_t part[SCAN_THREADS / 64];
    int32_t s = 0;
    for (int64_t k = threadIdx.x; k < m; k += SCAN_THREADS)
        s += a[k];
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = s;
    __syncthreads();
    int32_t tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w)
        tot += part[w];
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------- host side

Grid make_grid(const ib_level* lv);
int check_level(const ib_level* lv);
void set_hip_error(hipError_t e);
int launch_status();

// Device-wide exclusive scan of int32 (in may alias out).  total (device,
// nullable) receives the sum.  Workspace bytes from scan_workspace(n).
size_t scan_workspace(int64_t n);
// With shift > 0 the scanned values are in[i] >> shift.
void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* ws,
                    hipStream_t st, int shift = 0);

// Exclusive scans of two int32 arrays of the same length (outputs may alias
// inputs); totals (device, nullable).  Workspace bytes from scan2_workspace(n).
size_t scan2_workspace(int64_t n);
void scan_exclusive2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1,
                     int64_t n, int32_t* total0, int32_t* total1, void* ws, hipStream_t st);

// Stable LSD radix sort of (key, val) int32 pairs on the low `bits` bits of
// the key.  n_dev (device, nullable) holds the live count <= n_max.  Result
// is left in (keys, vals); (tk, tv) are scratch of n_max entries.
size_t radix_workspace(int64_t n_max);
void radix_sort_pairs(int32_t* keys, int32_t* vals, int32_t* tk, int32_t* tv, int64_t n_max,
                      const int32_t* n_dev, int bits, void* ws, hipStream_t st);

// offs[t] = first i with (keys[i] & mask) >= t, t = 0..T (masked keys sorted
// ascending).
void lower_bounds(const int32_t* keys, int64_t n_max, const int32_t* n_dev, int32_t* offs,
                  int64_t T, hipStream_t st, int32_t mask = -1);

inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Outputs of a call set to NaN when its bucket set is flagged (flag[0] or
// flag[1] nonzero on the device): up to two fields in the box layout (valid
// cells only), two vectors in the field precision and four FP64 vectors.
// Enqueue-only; no host synchronization.
struct PoisonSet {
    void* field[2] = {nullptr, nullptr};
    void* vec[2] = {nullptr, nullptr};
    int64_t nvec[2] = {0, 0};
    double* dvec[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t ndvec[4] = {0, 0, 0, 0};
};
void poison_if_flagged(const int32_t* flag, const Grid& g, ib_prec prec, const PoisonSet& ps,
                       hipStream_t st);

// Kernel classes timed by the optional per-plan profiler (see ib_plan_profile).
enum ProfKind {
    PK_PREP = 0, PK_LISTS, PK_INTERP_U0, PK_SPREAD, PK_INTERP_G, PK_SPREAD_FINAL, PK_FILL,
    PK_UNSORT, PK_RESID, PK_COUNT
};

// Start/stop HIP events around launches on the caller's stream; read back
// (after the stream has passed them) into per-class totals.
struct Profiler {
    static constexpr int MAXP = 1024;
    hipEvent_t ev[2 * MAXP];
    int kind[MAXP];
    int n = 0, created = 0, dropped = 0;
    double total_ms[PK_COUNT] = {};
    int64_t calls[PK_COUNT] = {};
    int open = -1;
    int init();
    void begin(int k, hipStream_t st);
    void end(hipStream_t st);
    int collect();
    void release();
};

// Bump allocator over a caller workspace.
struct Carver {
    char* p;
    size_t used, cap;
    explicit Carver(void* base, size_t c) : p((char*)base), used(0), cap(c) {}
    template <typename U>
    U* take(size_t count)
    {
        U* r = (U*)(p ? p + used : nullptr);
        used += align_up(sizeof(U) * (count ? count : 1));
        return r;
    }
    bool ok() const { return used <= cap; }
};

}  // namespace ibx
