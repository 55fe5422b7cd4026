// batched.hip -- the batched path of Algorithm 1 for many particles at once.
//
// The interpolation operator is linear, so with G^m = S F^m (the force field
// before the dt factor) the velocity at the markers in iteration m+1 is
//     J u^(m) = J u0 + dt J G^m.
// J u0 is formed once (first iteration); later iterations move only marker
// data and G, never the velocity field:
//     D     = (U^d - J u0)/dt,   F^1 = D,
//     F^m   = F^(m-1) + D - J G^(m-1),          m = 2..ns,
//     f     = G^ns,  ustar = u0 + dt G^ns.
// This is the recurrence of Algorithm 1 with the correction substituted into
// the next interpolation; results equal the literal loop up to rounding.
//
// Markers are processed in bucket order (sorted by owning 8^3 tile).  Each
// marker's stencil is precomputed once per call into a 64-byte (FP32) record
// -- stencil base relative to its owning tile's frame, P weights per axis,
// dV/h^3 -- and its force is kept as one 4-vector, so the spreading kernel's
// gathers of a source touch one or two cache lines.  U^d and D stay as
// structure-of-arrays (read only by the marker's own interpolation item).
//
// Kernels (persistent workgroups striding over device-side work lists; see
// tiles.h for the two hot ones):
//   interp   work item = up to bw markers of one tile; tile + halo of u0 or G
//            staged in LDS, one thread per marker.
//   spread   work item = one tile with a non-empty source list; one wavefront,
//            lane = (y, z) row of the tile accumulated in registers.  Result
//            to the compact per-tile G slots.
//   finalize f and ustar = u0 + dt G on every valid cell of the covered boxes,
//            box-wide rows per workgroup.  No float atomics anywhere.
#include "paths.h"

namespace ibx {

template <int P>
struct Halo {
    static constexpr int g = P == 4 ? 2 : 1;
    static constexpr int R = TILE + 2 * g;
    static constexpr int R3 = R * R * R;
};

struct Item {
    int32_t tile, start, count, pad;
};

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

// Stencil record of one marker (sorted order), read by every work item
// that the marker touches: geo = (r_x, r_y, r_z, dV/h^3) with r_a the offset
// s_a - b_a - 1/2 of the grid coordinate from the stencil's first cell
// centre (the weights follow from it, axis_weights_r), and the stencil base
// in the owning-tile frame (wrapped owning cell + (b - floor(s))) packed in
// 21-bit fields, each biased by RB_BIAS.
constexpr int RB_BITS = 21, RB_BIAS = 4;
constexpr int64_t RB_MASK = (int64_t(1) << RB_BITS) - 1;

__device__ inline void unpack_rb(int64_t v, int* rb)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        rb[a] = (int)((v >> (RB_BITS * a)) & RB_MASK) - RB_BIAS;
}

// The P weights of one axis from r = s - b - 1/2.  With d = r - 1 the
// distances to the P stencil points are 1 + d, |d|, 1 - d (and 2 - d), each
// on a fixed branch of the kernel, and all branches share one square root.
// P = 4: r in [1, 2), phi = (3 - 2|x| + q)/8 or (5 - 2|x| - q')/8 with
// q^2 = 1 + 4d - 4d^2; P = 3: r in [1/2, 3/2), q^2 = 1 - 3d^2.
__device__ inline float root(float x)
{
    return __builtin_amdgcn_sqrtf(x);   // the hardware square root (1 ulp), x in [1/4, 2]
}

__device__ inline double root(double x)
{
    return sqrt(x);
}

template <typename T, int P>
__device__ inline void axis_weights_r(T r, T* w)
{
    const T d = r - T(1);
    if (P == 4) {
        const T q = root(T(1) + T(4) * d * (T(1) - d)) * T(0.125);
        const T a = T(0.375) - T(0.25) * d, b = T(0.125) + T(0.25) * d;
        w[0] = a - q;
        w[1] = a + q;
        w[2] = b + q;
        w[3] = b - q;
    } else {
        const T q = root(T(1) - T(3) * d * d);
        const T q6 = q * T(1.0 / 6.0);
        w[0] = T(1.0 / 3.0) - T(0.5) * d - q6;
        w[1] = T(1.0 / 3.0) + T(1.0 / 3.0) * q;
        w[P - 1] = T(1.0 / 3.0) + T(0.5) * d - q6;
    }
}

// The same P weights and their derivatives with respect to r (= with respect
// to the grid coordinate s; divide by h for the derivative in X).  P = 4:
// dq/dd = (1 - 2d)/(4 sqrt(1 + 4d - 4d^2)); P = 3: dq/dd = -3d/q.  The roots
// stay away from zero on these branches (1 + 4d - 4d^2 >= 1, 1 - 3d^2 >= 1/4).
template <typename T, int P>
__device__ inline void axis_weights_rd(T r, T* w, T* dw)
{
    const T d = r - T(1);
    if (P == 4) {
        const T S = root(T(1) + T(4) * d * (T(1) - d));
        const T q = S * T(0.125);
        const T dq = (T(1) - T(2) * d) / (T(4) * S);
        const T a = T(0.375) - T(0.25) * d, b = T(0.125) + T(0.25) * d;
        w[0] = a - q;
        w[1] = a + q;
        w[2] = b + q;
        w[3] = b - q;
        dw[0] = T(-0.25) - dq;
        dw[1] = T(-0.25) + dq;
        dw[2] = T(0.25) + dq;
        dw[3] = T(0.25) - dq;
    } else {
        const T q = root(T(1) - T(3) * d * d);
        const T q6 = q * T(1.0 / 6.0);
        const T dq = T(-3) * d / q;
        w[0] = T(1.0 / 3.0) - T(0.5) * d - q6;
        w[1] = T(1.0 / 3.0) + T(1.0 / 3.0) * q;
        w[P - 1] = T(1.0 / 3.0) + T(0.5) * d - q6;
        dw[0] = T(-0.5) - dq * T(1.0 / 6.0);
        dw[1] = dq * T(1.0 / 3.0);
        dw[P - 1] = T(0.5) - dq * T(1.0 / 6.0);
    }
}

template <typename T>
struct MarkerData {
    typename Vec4<T>::type* geo;      // [n] (r_x, r_y, r_z, dV/h^3)
    int64_t* rb;                      // [n] packed stencil base
    typename Vec4<T>::type* f4;       // [n] F^m (x, y, z, 0)
    T* ud;                            // [3][n] U^d
    T* d;                             // [3][n] D = (U^d - J u0)/dt
};

__device__ inline void tile_coords(const Grid& g, int t, int* lo)
{
    lo[0] = (t % g.nt[0]) * TILE;
    lo[1] = ((t / g.nt[0]) % g.nt[1]) * TILE;
    lo[2] = (t / (g.nt[0] * g.nt[1])) * TILE;
}

// Box-layout element offset of a tile's first cell (a tile never straddles
// boxes: the box edge is a multiple of 8), or -1 in an uncovered box.
__device__ inline int64_t tile_base(const Grid& g, const int* lo)
{
    const int bx = lo[0] / g.box, by = lo[1] / g.box, bz = lo[2] / g.box;
    const int id = g.lut[bx + g.nb[0] * (by + g.nb[1] * bz)];
    if (id < 0)
        return -1;
    return (int64_t)id * g.bstride +
           ((int64_t)(lo[2] - bz * g.box + g.ngrow) * g.ext + (lo[1] - by * g.box + g.ngrow)) *
               g.ext +
           (lo[0] - bx * g.box + g.ngrow);
}

// ------------------------------------------------------------------ prep

// Record and U^d of the marker at sorted position i.
template <typename T, int P>
__device__ inline void prep_marker(int64_t i, const Grid& g, int64_t nl,
                                   const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, const int32_t* __restrict__ pid,
                                   const double* __restrict__ dv, const int32_t* __restrict__ perm,
                                   const double* __restrict__ xc, const double* __restrict__ up,
                                   const double* __restrict__ om, const MarkerData<T>& s)
{
    if (i >= nl)
        return;
    const int64_t l = perm[i];
    const double X[3] = {x[l], y[l], z[l]};
    T r[3];
    int64_t pk = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double sa = grid_coord(g, a, X[a]);
        const int b = stencil_base<P>(sa);
        r[a] = (T)(sa - (double)b - 0.5);
        const int fl = (int)floor(sa);
        int c = fl;
        if (g.periodic[a]) {
            // markers sit at most a period outside: one add or subtract, else the modulo
            c = c < 0 ? c + g.n[a] : (c >= g.n[a] ? c - g.n[a] : c);
            if ((unsigned)c >= (unsigned)g.n[a])
                c = wrapi(fl, g.n[a]);
        }
        pk |= (int64_t)(c + (b - fl) + RB_BIAS) << (RB_BITS * a);
    }
    const int p = pid[l];
    typename Vec4<T>::type q;
    q.x = r[0];
    q.y = r[1];
    q.z = r[2];
    q.w = (T)(dv[p] * g.inv_h3);
    s.geo[i] = q;
    s.rb[i] = pk;
    const double R0 = X[0] - xc[3 * p], R1 = X[1] - xc[3 * p + 1], R2 = X[2] - xc[3 * p + 2];
    const double w0 = om[3 * p], w1 = om[3 * p + 1], w2 = om[3 * p + 2];
    s.ud[0 * nl + i] = (T)(up[3 * p + 0] + (w1 * R2 - w2 * R1));
    s.ud[1 * nl + i] = (T)(up[3 * p + 1] + (w2 * R0 - w0 * R2));
    s.ud[2 * nl + i] = (T)(up[3 * p + 2] + (w0 * R1 - w1 * R0));
}

#include "tiles.h"

// ------------------------------------------------------------------ work lists

// Spreading order.  The active positions are cut into NXCD equal slabs, one
// per XCD (workgroups are dealt to the XCDs round-robin by id, and each XCD
// has its own L2, so neighbouring tiles -- which share source markers -- stay
// on one XCD); inside a slab they are ordered by decreasing source count, so
// that a static snake deal over the slab's workgroups gives each a similar
// load.  Cost bins (source count, clamped) are counted per block in LDS and
// then globally; the order inside a bin is whatever the atomics give, which
// moves no result (each tile is summed by one wavefront in its own fixed
// order and stored to its own slot).
constexpr int COST_BINS = 256;

__device__ inline int slab_of(int a, int n_act)
{
    const int per = (n_act + NXCD - 1) / NXCD;
    return a / per;
}

// Markers of the interpolation work tile that tile t leads (first one in
// *start): tile t alone, or with PAIR (work tiles of two x neighbours) tiles
// t and t + 1 when t has an even x index (t alone when it ends its row), and
// none when its x index is odd.  Markers are sorted by tile, so the two
// tiles' markers are one run.  (Tile indices fit 32 bits: the marker offsets
// are 32-bit.)
template <bool PAIR>
__device__ inline int item_markers(const int32_t* __restrict__ tile_offs, int64_t t, int nt0,
                                   int* start)
{
    const int s = tile_offs[t];
    *start = s;
    if (!PAIR)
        return tile_offs[t + 1] - s;
    const int tx = (int)t % nt0;
    if (tx & 1)
        return 0;
    return (tx + 1 < nt0 ? tile_offs[t + 2] : tile_offs[t + 1]) - s;
}

// The interpolation items of work tile t, from its first item io on.
template <bool PAIR>
__device__ inline void write_items(int64_t t, int io, int bw, int nt0,
                                   const int32_t* __restrict__ tile_offs, Item* items)
{
    int start;
    const int cnt = item_markers<PAIR>(tile_offs, t, nt0, &start);
    for (int k = 0; k * bw < cnt; ++k) {
        Item it;
        it.tile = (int32_t)t;
        it.start = start + k * bw;
        it.count = min(bw, cnt - k * bw);
        it.pad = 0;
        items[io + k] = it;
    }
}

// Block blk of 256 threads (block 0 also clears the cost histogram that
// k_cost_hist fills next).
template <bool PAIR>
__device__ inline void tile_counts_block(unsigned blk, int64_t T, int bw, int nt0,
                                         const int32_t* __restrict__ tile_offs,
                                         const int32_t* __restrict__ src_offs, int32_t* item_cnt,
                                         int32_t* act, int32_t* __restrict__ hist)
{
    if (blk == 0)
        for (int b = threadIdx.x; b < NXCD * COST_BINS; b += 256)
            hist[b] = 0;
    const int64_t t = (int64_t)blk * 256 + threadIdx.x;
    if (t >= T)
        return;
    int start;
    const int cnt = item_markers<PAIR>(tile_offs, t, nt0, &start);
    item_cnt[t] = (cnt + bw - 1) / bw;
    act[t] = src_offs[t + 1] > src_offs[t] ? 1 : 0;
}

// hist[x][b]: active tiles of slab x in cost bin b (zeroed beforehand); and
// the interpolation items of every work tile.
template <bool PAIR>
__global__ void __launch_bounds__(256)
k_cost_hist(int64_t T, const int32_t* __restrict__ src_offs, const int32_t* __restrict__ act_offs,
            const int32_t* __restrict__ nactive, int32_t* __restrict__ hist, int bw, int nt0,
            const int32_t* __restrict__ tile_offs, const int32_t* __restrict__ item_offs,
            Item* items)
{
    __shared__ int32_t lh[NXCD * COST_BINS];
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        lh[b] = 0;
    __syncthreads();
    const int n_act = *nactive;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) {
        const int c = src_offs[t + 1] - src_offs[t];
        if (c > 0)
            atomicAdd(&lh[slab_of(act_offs[t], n_act) * COST_BINS + min(c, COST_BINS - 1)], 1);
        write_items<PAIR>(t, item_offs[t], bw, nt0, tile_offs, items);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        if (lh[b])
            atomicAdd(&hist[b], lh[b]);
}

// The two work-list scans for grids of at most SCAN_FUSE / 2 scan tiles, in
// two passes.  Pass 1 (blocks of SCAN_THREADS threads): block id = b < nb
// scans the interpolation item counts ceil(markers / bw) of scan tile b,
// block nb + b the flags "source list not empty" (the inputs are formed from
// the offsets on the fly); block 0 also clears the cost histogram.
template <bool PAIR>
__device__ inline void list_scan_block(unsigned id, int64_t T, int bw, int nt0,
                                       const int32_t* __restrict__ tile_offs,
                                       const int32_t* __restrict__ src_offs,
                                       int32_t* __restrict__ item_offs,
                                       int32_t* __restrict__ act_offs, int32_t* __restrict__ sums,
                                       int32_t* __restrict__ hist)
{
    __shared__ int32_t ts[SCAN_THREADS];
    if (id == 0)
        for (int b = threadIdx.x; b < NXCD * COST_BINS; b += SCAN_THREADS)
            hist[b] = 0;
    const int64_t nb = (T + SCAN_TILE - 1) / SCAN_TILE;
    const bool second = id >= nb;
    const int64_t blk = second ? id - nb : id;
    int32_t* out = second ? act_offs : item_offs;
    const int t = threadIdx.x;
    const int64_t base = blk * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + k;
        v[k] = 0;
        if (i < T) {
            int start;
            v[k] = second ? (src_offs[i + 1] > src_offs[i] ? 1 : 0)
                          : (item_markers<PAIR>(tile_offs, i, nt0, &start) + bw - 1) / bw;
        }
        tsum += v[k];
    }
    ts[t] = tsum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const int32_t x = t >= off ? ts[t - off] : 0;
        __syncthreads();
        ts[t] += x;
        __syncthreads();
    }
    int32_t run = ts[t] - tsum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < T)
            out[base + k] = run;
        run += v[k];
    }
    if (t == SCAN_THREADS - 1)
        sums[id] = ts[t];
}

// Pass 2: each workgroup adds the totals of the scan tiles before its own
// (for the flags, less the item total), the last one of each array writes its
// total (nitems, nactive), and the flag workgroups count their spreading
// tiles into the cost histogram (as k_cost_hist does); the item workgroups
// also write the interpolation items of their work tiles.
template <bool PAIR>
__global__ void __launch_bounds__(SCAN_THREADS)
k_list_add(int64_t T, const int32_t* __restrict__ src_offs, int32_t* __restrict__ item_offs,
           int32_t* __restrict__ act_offs, const int32_t* __restrict__ sums,
           int32_t* __restrict__ nitems, int32_t* __restrict__ nactive,
           int32_t* __restrict__ hist, int bw, int nt0, const int32_t* __restrict__ tile_offs,
           Item* items)
{
    __shared__ int32_t lh[NXCD * COST_BINS];
    const int64_t nb = (T + SCAN_TILE - 1) / SCAN_TILE;
    const bool second = blockIdx.x >= nb;
    const int64_t blk = second ? blockIdx.x - nb : blockIdx.x;
    int32_t* out = second ? act_offs : item_offs;
    const int32_t pre = group_sum(sums, blockIdx.x);
    const int32_t first_total = group_sum(sums, nb);
    const int32_t n_act = group_sum(sums + nb, nb);
    const int32_t add = pre - (second ? first_total : 0);
    const int64_t base = blk * SCAN_TILE;
    if (threadIdx.x == 0 && blk == nb - 1) {
        if (second)
            *nactive = n_act;
        else
            *nitems = first_total;
    }
    if (!second) {
        for (int k = threadIdx.x; k < SCAN_TILE; k += blockDim.x)
            if (base + k < T) {
                const int io = out[base + k] + add;
                out[base + k] = io;
                write_items<PAIR>(base + k, io, bw, nt0, tile_offs, items);
            }
        return;
    }
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        lh[b] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < SCAN_TILE; k += blockDim.x) {
        const int64_t i = base + k;
        if (i < T) {
            const int32_t a = out[i] + add;
            out[i] = a;
            const int c = src_offs[i + 1] - src_offs[i];
            if (c > 0)
                atomicAdd(&lh[slab_of(a, n_act) * COST_BINS + min(c, COST_BINS - 1)], 1);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        if (lh[b])
            atomicAdd(&hist[b], lh[b]);
}

// The marker records and the first work-list pass, which are independent,
// in one launch of 256-thread blocks: blocks below nlist run the list pass
// (SCAN: the fused list scan over 2 nb blocks; else the tile counts), the
// others form the records, one thread per marker in bucket order.
template <typename T, int P, bool PAIR, bool SCAN>
__global__ void __launch_bounds__(256)
k_prep_lists(unsigned nlist, Grid g, int64_t nl, const double* __restrict__ x,
             const double* __restrict__ y, const double* __restrict__ z,
             const int32_t* __restrict__ pid, const double* __restrict__ dv,
             const int32_t* __restrict__ perm, const double* __restrict__ xc,
             const double* __restrict__ up, const double* __restrict__ om, MarkerData<T> s,
             int bw, const int32_t* __restrict__ tile_offs, const int32_t* __restrict__ src_offs,
             int32_t* __restrict__ out_items, int32_t* __restrict__ out_act,
             int32_t* __restrict__ sums, int32_t* __restrict__ hist)
{
    static_assert(SCAN_THREADS == 256, "one block size for both parts");
    if (blockIdx.x >= nlist) {
        prep_marker<T, P>((int64_t)(blockIdx.x - nlist) * 256 + threadIdx.x, g, nl, x, y, z,
                          pid, dv, perm, xc, up, om, s);
        return;
    }
    if constexpr (SCAN)
        list_scan_block<PAIR>(blockIdx.x, g.ntiles, bw, g.nt[0], tile_offs, src_offs, out_items,
                              out_act, sums, hist);
    else
        tile_counts_block<PAIR>(blockIdx.x, g.ntiles, bw, g.nt[0], tile_offs, src_offs,
                                out_items, out_act, hist);
}

// cur[x][b] = first position of slab x plus its tiles in bins above b (slab
// x = blk, thread b of COST_BINS).
__device__ inline void bin_scan_block(unsigned blk, const int32_t* __restrict__ hist,
                                      const int32_t* __restrict__ nactive,
                                      int32_t* __restrict__ cur)
{
    __shared__ int32_t v[COST_BINS];
    const int b = threadIdx.x, x = (int)blk;
    const int per = (*nactive + NXCD - 1) / NXCD;
    const int32_t* h = hist + x * COST_BINS;
    v[b] = h[COST_BINS - 1 - b];
    __syncthreads();
    for (int o = 1; o < COST_BINS; o <<= 1) {
        const int add = b >= o ? v[b - o] : 0;
        __syncthreads();
        v[b] += add;
        __syncthreads();
    }
    // inclusive over reversed bins -> exclusive start of bin COST_BINS-1-b
    cur[x * COST_BINS + COST_BINS - 1 - b] = x * per + v[b] - h[COST_BINS - 1 - b];
}

// The cost-bin scan and the items' neighbour offsets, which do not depend on
// each other, in one launch of COST_BINS-thread blocks: blocks below NXCD
// scan the bins of one slab each, the others take one (item, neighbour)
// each ([it][9 NBX] into nb_u and nb_g; the items are written by then).
template <bool PAIR>
__global__ void __launch_bounds__(COST_BINS)
k_bins_bases(const int32_t* __restrict__ hist, const int32_t* __restrict__ nactive,
             int32_t* __restrict__ cur, Grid g, const Item* __restrict__ items,
             const int32_t* __restrict__ nitems, const int32_t* __restrict__ src_offs,
             const int32_t* __restrict__ act_offs, int64_t* __restrict__ nb_u,
             int64_t* __restrict__ nb_g)
{
    static_assert(COST_BINS == 256, "one block size for both parts");
    if (blockIdx.x < NXCD) {
        bin_scan_block(blockIdx.x, hist, nactive, cur);
        return;
    }
    constexpr int NBX = PAIR ? 4 : 3, NNB = 9 * NBX;
    const int64_t q = (int64_t)(blockIdx.x - NXCD) * COST_BINS + threadIdx.x;
    const int64_t it = q / NNB;
    if (it >= *nitems)
        return;
    int64_t bu, bg;
    item_base<NBX>(g, items[it].tile, (int)(q - it * NNB), src_offs, act_offs, &bu, &bg);
    nb_u[q] = bu;
    nb_g[q] = bg;
}

// Work lists: the G slot of every tile (-1 when its source list is empty),
// and the spreading entries (slot, tile, source range) in spreading order
// (cur[x][b] holds the first free position of bin b of slab x).
__global__ void __launch_bounds__(256)
k_fill_lists(int64_t T, const int32_t* __restrict__ src_offs,
             const int32_t* __restrict__ act_offs, const int32_t* __restrict__ nactive,
             int32_t* slot, int32_t* __restrict__ cur, int4* __restrict__ sent)
{
    __shared__ int32_t lc[NXCD * COST_BINS];
    __shared__ int32_t base[NXCD * COST_BINS];
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        lc[b] = 0;
    __syncthreads();
    const int n_act = *nactive;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bin = -1, rank = 0, s0 = 0, s1 = 0;
    if (t < T) {
        s0 = src_offs[t];
        s1 = src_offs[t + 1];
        const int c = s1 - s0;
        if (c > 0) {
            const int a = act_offs[t];
            slot[t] = a;
            bin = slab_of(a, n_act) * COST_BINS + min(c, COST_BINS - 1);
            rank = atomicAdd(&lc[bin], 1);
        } else {
            slot[t] = -1;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NXCD * COST_BINS; b += blockDim.x)
        if (lc[b])
            base[b] = atomicAdd(&cur[b], lc[b]);
    __syncthreads();
    if (bin >= 0)
        sent[base[bin] + rank] = make_int4(act_offs[t], (int)t, s0, s1);
}


// Persistent grid of a tile kernel: the workgroups that can be resident at
// once (optionally capped per CU), a multiple of 8 for the XCD split.
template <auto K, int BLOCK>
int resident_grid(int ncu, int cap)
{
    static const int fit = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, K, BLOCK, 0) != hipSuccess || n < 1)
            n = 1;
        return n;
    }();
    const int per_cu = cap > 0 && cap < fit ? cap : fit;
    const int grid = ncu * per_cu / NXCD * NXCD;
    return grid > NXCD ? grid : NXCD;
}

// ------------------------------------------------------------------ fill

// NaN in ustar and f (either nullable) on every valid cell of the covered
// boxes and in Fp[0 .. nF): the finalize's outputs when the bucket set is
// flagged (an error path, so a plain grid-stride loop).
template <typename T>
__device__ void finalize_poison(const Grid& g, T* ustar, T* f, T* Fp, int64_t nF)
{
    const T nan = (T)__builtin_nan("");
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_box = (int64_t)g.box * g.box * g.box;
    for (int64_t q = t0; (ustar || f) && q < per_box * g.nbox; q += stride) {
        const int64_t bid = q / per_box, r = q - bid * per_box;
        const int lx = (int)(r % g.box) + g.ngrow;
        const int ly = (int)((r / g.box) % g.box) + g.ngrow;
        const int lz = (int)(r / ((int64_t)g.box * g.box)) + g.ngrow;
        const int64_t off = bid * g.bstride + ((int64_t)lz * g.ext + ly) * g.ext + lx;
        for (int c = 0; c < 3; ++c) {
            if (ustar)
                ustar[off + c * g.cstride] = nan;
            if (f)
                f[off + c * g.cstride] = nan;
        }
    }
    for (int64_t i = t0; Fp && i < nF; i += stride)
        Fp[i] = nan;
}

// Last step of Algorithm 1 on every valid cell of the covered boxes:
// f = G^ns and ustar = u0 + dt G^ns, with G = 0 on tiles no marker reaches
// (and everywhere when use_g is 0) and on the slot rows whose bit in the
// tile's row mask (tilemask, indexed by tile) is clear.  One workgroup per
// (box, row of tiles in y, z plane): box-wide x rows, so the box layout is
// written in long runs.
// In place (ustar == u0) only the cells whose force is not exactly zero are
// read and rewritten (u0 + dt 0 = u0): inside the tiles that have a force
// slot, most cells lie outside every stencil.  With f_acc, f += G^ns instead,
// on the same cells.  ustar may be null (f only).  A separate ustar takes u0
// on the cells without force (copy).  With flag (nullable) raised (a flagged
// bucket set), f and ustar are NaN on every such cell instead, and so is
// Fp[0 .. nF) (the marker forces, written before this kernel).
template <typename T, bool F_ACC, bool MASK>
__global__ void __launch_bounds__(256)
k_finalize(Grid g, const int32_t* __restrict__ slot, const T* __restrict__ G,
           const uint64_t* __restrict__ tilemask, const T* u0, T* ustar, T* __restrict__ f,
           double dt, int use_g, int copy, const int32_t* __restrict__ flag, T* __restrict__ Fp,
           int64_t nF)
{
    if (flag && (flag[0] | flag[1]) != 0) {
        finalize_poison(g, ustar, f, Fp, nF);
        return;
    }
    __shared__ int tslot[64];                 // G slot of each tile along the row
    __shared__ uint64_t tmask[64];            // and its row mask
    const int B = g.box;
    const int nty = B / TILE, ntx = B / TILE;
    const int64_t items = (int64_t)g.nbox * nty * B;
    const T tdt = (T)dt;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int bid = (int)(it / ((int64_t)nty * B));
        const int rem = (int)(it - (int64_t)bid * nty * B);
        const int ty = rem / B, lz = rem - ty * B;
        const int bx0 = g.box_lo[3 * bid], by0 = g.box_lo[3 * bid + 1], bz0 = g.box_lo[3 * bid + 2];
        const int cz = bz0 + lz, cyt = (by0 >> 3) + ty;
        for (int k = threadIdx.x; k < ntx; k += blockDim.x) {
            const int64_t tk = (bx0 >> 3) + k + g.nt[0] * (cyt + g.nt[1] * (cz >> 3));
            tslot[k] = use_g ? slot[tk] : -1;
            if (MASK)
                tmask[k] = use_g ? tilemask[tk] : 0ull;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < TILE * B; q += blockDim.x) {
            const int yy = q / B, lx = q - yy * B;
            const int ly = ty * TILE + yy;
            const int s =
                !MASK || (tmask[lx >> 3] >> (yy + TILE * (cz & 7))) & 1 ? tslot[lx >> 3] : -1;
            const int64_t off = (int64_t)bid * g.bstride +
                                ((int64_t)(lz + g.ngrow) * g.ext + (ly + g.ngrow)) * g.ext +
                                (lx + g.ngrow);
            const int64_t go =
                (int64_t)s * 3 * TILE_CELLS + (lx & 7) + TILE * (yy + TILE * (cz & 7));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T v = s >= 0 ? G[go + c * TILE_CELLS] : T(0);
                const int64_t o = off + c * g.cstride;
                // streaming stores: nothing here is read again by this kernel
                if (f && !F_ACC)
                    __builtin_nontemporal_store(v, &f[o]);
                else if (f && v != T(0))
                    f[o] += v;
                if (!ustar)
                    continue;
                if (v != T(0))
                    __builtin_nontemporal_store(u0[o] + tdt * v, &ustar[o]);
                else if (copy)
                    __builtin_nontemporal_store(u0[o], &ustar[o]);
            }
        }
        __syncthreads();
    }
}

template <typename T>
struct Pair;
template <>
struct Pair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// The same for an even ghost width, two neighbouring x cells per thread (every
// pair starts on an even element of the box layout and of the tile slots):
// one workgroup per (box, row of tiles in y, pair of z planes).
template <typename T, bool F_ACC, bool MASK>
__global__ void __launch_bounds__(256)
k_finalize_pairs(Grid g, const int32_t* __restrict__ slot, const T* __restrict__ G,
                 const uint64_t* __restrict__ tilemask, const T* u0, T* ustar, T* __restrict__ f,
                 double dt, int use_g, int copy, const int32_t* __restrict__ flag,
                 T* __restrict__ Fp, int64_t nF)
{
    using V2 = typename Pair<T>::type;
    if (flag && (flag[0] | flag[1]) != 0) {
        finalize_poison(g, ustar, f, Fp, nF);
        return;
    }
    __shared__ int tslot[64];                 // G slot of each tile along the row
    __shared__ uint64_t tmask[64];            // and its row mask
    const int B = g.box;
    const int nty = B / TILE, ntx = B / TILE, npx = B / 2;
    const int per_box = nty * (B / 2);
    const int64_t items = (int64_t)g.nbox * per_box;
    const T tdt = (T)dt;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int bid = (int)(it / per_box);
        const int rem = (int)(it - (int64_t)bid * per_box);
        const int ty = rem / (B / 2), lz0 = 2 * (rem - ty * (B / 2));
        const int bx0 = g.box_lo[3 * bid], by0 = g.box_lo[3 * bid + 1], bz0 = g.box_lo[3 * bid + 2];
        const int cz0 = bz0 + lz0, cyt = (by0 >> 3) + ty;
        for (int k = threadIdx.x; k < ntx; k += blockDim.x) {
            const int64_t tk = (bx0 >> 3) + k + g.nt[0] * (cyt + g.nt[1] * (cz0 >> 3));
            tslot[k] = use_g ? slot[tk] : -1;
            if (MASK)
                tmask[k] = use_g ? tilemask[tk] : 0ull;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * TILE * npx; q += blockDim.x) {
            const int px = q % npx, r = q / npx;
            const int yy = r & (TILE - 1), pz = r >> 3;
            const int lx = 2 * px, ly = ty * TILE + yy, lz = lz0 + pz;
            const int s = !MASK || (tmask[lx >> 3] >> (yy + TILE * ((cz0 + pz) & 7))) & 1
                              ? tslot[lx >> 3]
                              : -1;
            const int64_t off = (int64_t)bid * g.bstride +
                                ((int64_t)(lz + g.ngrow) * g.ext + (ly + g.ngrow)) * g.ext +
                                (lx + g.ngrow);
            const int64_t go =
                (int64_t)s * 3 * TILE_CELLS + (lx & 7) + TILE * (yy + TILE * ((cz0 + pz) & 7));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                V2 v = {T(0), T(0)};
                if (s >= 0)
                    v = *reinterpret_cast<const V2*>(G + go + c * TILE_CELLS);
                const int64_t o = off + c * g.cstride;
                // in place, a pair without force keeps u0 and needs no traffic
                const bool force = v.x != T(0) || v.y != T(0);
                if (f && !F_ACC) {
                    __builtin_nontemporal_store(v, reinterpret_cast<V2*>(f + o));
                } else if (f && force) {
                    V2 w = *reinterpret_cast<const V2*>(f + o);
                    *reinterpret_cast<V2*>(f + o) = w + v;
                }
                if (!ustar) {
                } else if (force) {
                    const V2 a = *reinterpret_cast<const V2*>(u0 + o);
                    __builtin_nontemporal_store(a + tdt * v, reinterpret_cast<V2*>(ustar + o));
                } else if (copy) {
                    const V2 a = *reinterpret_cast<const V2*>(u0 + o);
                    __builtin_nontemporal_store(a, reinterpret_cast<V2*>(ustar + o));
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, bool F_ACC, bool MASK>
static void finalize_kernel(bool pairs, unsigned grid, unsigned gp, hipStream_t st, const Grid& g,
                            const int32_t* slot, const T* G, const uint64_t* tilemask,
                            const T* u0, T* ustar, T* f, double dt, int use_g, int copy,
                            const int32_t* flag, T* Fp, int64_t nF)
{
    if (pairs)
        k_finalize_pairs<T, F_ACC, MASK><<<gp, 256, 0, st>>>(g, slot, G, tilemask, u0, ustar, f,
                                                             dt, use_g, copy, flag, Fp, nF);
    else
        k_finalize<T, F_ACC, MASK><<<grid, 256, 0, st>>>(g, slot, G, tilemask, u0, ustar, f, dt,
                                                         use_g, copy, flag, Fp, nF);
}

// With flag, the kernel also stands in for the flag check of the outputs
// (ustar, f and Fp[0 .. nF)).
template <typename T>
static void launch_finalize(unsigned grid, hipStream_t st, const Grid& g, const int32_t* slot,
                            const T* G, const uint64_t* tilemask, const T* u0, T* ustar, T* f,
                            double dt, int use_g, int f_acc, int masks,
                            const int32_t* flag = nullptr, T* Fp = nullptr, int64_t nF = 0)
{
    const int copy = ustar && ustar != u0;
    // pairs of cells: rows start on even elements when ngrow is even, and the
    // pair loads and stores need the fields aligned to two elements
    const uintptr_t am = 2 * sizeof(T) - 1;
    const bool pairs = (g.ngrow & 1) == 0 && !((uintptr_t)u0 & am) &&
                       !((uintptr_t)ustar & am) && !((uintptr_t)f & am);
    const int64_t items = (int64_t)g.nbox * (g.box / TILE) * (g.box / 2);
    const unsigned gp = (unsigned)(items < 65535 ? (items > 0 ? items : 1) : 65535);
    if (f_acc && masks)
        finalize_kernel<T, true, true>(pairs, grid, gp, st, g, slot, G, tilemask, u0, ustar, f,
                                       dt, use_g, copy, flag, Fp, nF);
    else if (f_acc)
        finalize_kernel<T, true, false>(pairs, grid, gp, st, g, slot, G, tilemask, u0, ustar, f,
                                        dt, use_g, copy, flag, Fp, nF);
    else if (masks)
        finalize_kernel<T, false, true>(pairs, grid, gp, st, g, slot, G, tilemask, u0, ustar, f,
                                        dt, use_g, copy, flag, Fp, nF);
    else
        finalize_kernel<T, false, false>(pairs, grid, gp, st, g, slot, G, tilemask, u0, ustar, f,
                                         dt, use_g, copy, flag, Fp, nF);
}

template <typename T>
__global__ void k_unsort(int64_t nl, const int32_t* __restrict__ perm,
                         const typename Vec4<T>::type* __restrict__ f4, T* __restrict__ F)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl)
        return;
    const int64_t l = perm[i];
    const typename Vec4<T>::type v = f4[i];
    F[3 * l + 0] = v.x;
    F[3 * l + 1] = v.y;
    F[3 * l + 2] = v.z;
}

template <typename T>
__global__ void k_zero(int64_t n, T* a)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        a[q] = T(0);
}

// ------------------------------------------------------------------ host

// Neighbour tiles per interpolation item: 27 for an 8^3 work tile, 36 for a
// 16 x 8 x 8 one.
constexpr int NB_MAX = 36;

template <typename T>
struct BatchedWs {
    MarkerData<T> s;
    double* e2;
    double* part;
    Item* items;
    int32_t *item_cnt, *item_offs, *act, *act_offs, *slot, *nitems, *nactive;
    int32_t *hist, *cur;
    int4* sent;     // spreading order by decreasing cost: (slot, tile, sources begin, end)
    T* G;
    uint64_t* rmask;   // per slot: bit r set when row r of the slot is not all zeros
    uint64_t* tmask;   // the same per tile (stale on tiles without a slot)
    void* scan;
    int64_t max_items;
    int64_t *nb_u, *nb_g;   // [item][9 NBX] element offsets of the neighbouring tiles
};

template <typename T>
static BatchedWs<T> carve_batched(const Grid& g, int64_t nl, int bw, void* ws, size_t bytes,
                                  size_t* need)
{
    Carver cv(ws, bytes);
    BatchedWs<T> w;
    const int64_t T_ = g.ntiles;
    w.s.geo = cv.take<typename Vec4<T>::type>(nl);
    w.s.rb = cv.take<int64_t>(nl);
    w.s.f4 = cv.take<typename Vec4<T>::type>(nl);
    w.s.ud = cv.take<T>(3 * nl);
    w.s.d = cv.take<T>(3 * nl);
    w.e2 = cv.take<double>(nl);
    w.part = cv.take<double>(sum_partials(nl));
    w.max_items = T_ + nl / bw + 1;
    w.items = cv.take<Item>(w.max_items);
    w.item_cnt = cv.take<int32_t>(T_);
    w.item_offs = cv.take<int32_t>(T_);
    w.act = cv.take<int32_t>(T_);
    w.act_offs = cv.take<int32_t>(T_);
    w.hist = cv.take<int32_t>(NXCD * COST_BINS);
    w.cur = cv.take<int32_t>(NXCD * COST_BINS);
    w.sent = cv.take<int4>(T_);
    w.slot = cv.take<int32_t>(T_);
    w.nitems = cv.take<int32_t>(1);
    w.nactive = cv.take<int32_t>(1);
    const int64_t max_active = T_ < 8 * nl ? T_ : 8 * nl;
    w.G = cv.take<T>((size_t)3 * TILE_CELLS * (max_active > 0 ? max_active : 1));
    w.rmask = cv.take<uint64_t>(max_active > 0 ? max_active : 1);
    w.tmask = cv.take<uint64_t>(T_ > 0 ? T_ : 1);
    w.nb_u = cv.take<int64_t>(NB_MAX * w.max_items);
    w.nb_g = cv.take<int64_t>(NB_MAX * w.max_items);
    w.scan = cv.take<char>(scan2_workspace(T_));
    *need = cv.used;
    return w;
}

template <typename T, int P, int MODE, bool MASK, int TXW, int BW>
static void interp_kernel(const BatchedCfg& cfg, hipStream_t st, const Grid& g, int64_t nl,
                          double dt, const Item* items, const int32_t* nitems, const T* u0,
                          const T* G, const uint64_t* rmask, const int64_t* nbase,
                          const MarkerData<T>& s, double* e2, T* Fout, const int32_t* perm,
                          const T* vin, double* gX, int use_dv)
{
    constexpr auto K = k_interp_tiles<T, P, MODE, BW, MASK, TXW>;
    K<<<resident_grid<K, BW>(cfg.ncu, 0), BW, 0, st>>>(g, nl, dt, items, nitems, u0, G, nbase, s,
                                                       e2, Fout, perm, vin, gX, use_dv, rmask);
}

template <typename T, int P, int MODE, bool MASK, int TXW>
static void launch_interp_txw(const BatchedCfg& cfg, hipStream_t st, const Grid& g, int64_t nl,
                              double dt, const Item* items, const int32_t* nitems, const T* u0,
                              const T* G, const uint64_t* rmask, const int64_t* nbase,
                              const MarkerData<T>& s, double* e2, T* Fout, const int32_t* perm,
                              const T* vin, double* gX, int use_dv)
{
    if (cfg.bw == 64)
        interp_kernel<T, P, MODE, MASK, TXW, 64>(cfg, st, g, nl, dt, items, nitems, u0, G, rmask,
                                                 nbase, s, e2, Fout, perm, vin, gX, use_dv);
    else if (cfg.bw == 128)
        interp_kernel<T, P, MODE, MASK, TXW, 128>(cfg, st, g, nl, dt, items, nitems, u0, G,
                                                  rmask, nbase, s, e2, Fout, perm, vin, gX,
                                                  use_dv);
    else
        interp_kernel<T, P, MODE, MASK, TXW, 256>(cfg, st, g, nl, dt, items, nitems, u0, G,
                                                  rmask, nbase, s, e2, Fout, perm, vin, gX,
                                                  use_dv);
}

// Work tiles of two x neighbours are compiled for FP32 only (their halo in
// FP64 would need 69 KB of LDS).
template <typename T>
static int pair_items(const BatchedCfg& cfg)
{
    return sizeof(T) == 4 && cfg.txw == 2 * TILE;
}

template <typename T, int P, int MODE, bool MASK>
static void launch_interp_bw(const BatchedCfg& cfg, hipStream_t st, const Grid& g, int64_t nl,
                             double dt, const Item* items, const int32_t* nitems, const T* u0,
                             const T* G, const uint64_t* rmask, const int64_t* nbase,
                             const MarkerData<T>& s, double* e2, T* Fout, const int32_t* perm,
                             const T* vin, double* gX, int use_dv)
{
    if constexpr (sizeof(T) == 4) {
        if (pair_items<T>(cfg)) {
            launch_interp_txw<T, P, MODE, MASK, 2 * TILE>(cfg, st, g, nl, dt, items, nitems, u0,
                                                          G, rmask, nbase, s, e2, Fout, perm,
                                                          vin, gX, use_dv);
            return;
        }
    }
    launch_interp_txw<T, P, MODE, MASK, TILE>(cfg, st, g, nl, dt, items, nitems, u0, G, rmask,
                                              nbase, s, e2, Fout, perm, vin, gX, use_dv);
}

// Interpolation from the G slots (modes 1, 2) uses the slot row masks when the
// plan does.
template <typename T, int P, int MODE>
static void launch_interp(const BatchedCfg& cfg, hipStream_t st, const Grid& g, int64_t nl,
                          double dt, const Item* items, const int32_t* nitems, const T* u0,
                          const T* G, const uint64_t* rmask, const int64_t* nbase,
                          const MarkerData<T>& s, double* e2, T* Fout = nullptr,
                          const int32_t* perm = nullptr, const T* vin = nullptr,
                          double* gX = nullptr, int use_dv = 0)
{
    if constexpr (MODE == 1 || MODE == 2) {
        if (cfg.masks) {
            launch_interp_bw<T, P, MODE, true>(cfg, st, g, nl, dt, items, nitems, u0, G, rmask,
                                               nbase, s, e2, Fout, perm, vin, gX, use_dv);
            return;
        }
    }
    launch_interp_bw<T, P, MODE, false>(cfg, st, g, nl, dt, items, nitems, u0, G, rmask, nbase,
                                        s, e2, Fout, perm, vin, gX, use_dv);
}

// The tile spreading: one 2 x 2 x 2 block per lane for the 3-point kernel,
// one row per lane for the 4-point one (the faster layout for each width).
template <typename T, int P, bool MASK>
static void spread_kernel(const BatchedCfg& cfg, hipStream_t st, const Grid& g,
                          const BatchedWs<T>& w, const ib_buckets* b, int use_dv)
{
    if constexpr (P == 3) {
        constexpr auto K = k_spread_blocks<T, P, MASK>;
        K<<<resident_grid<K, 64>(cfg.ncu, cfg.wgs_s), 64, 0, st>>>(
            w.sent, w.nactive, b->src_idx, g, w.s, w.G, w.rmask, w.tmask, use_dv);
    } else {
        constexpr auto K = k_spread_tiles<T, P, MASK>;
        K<<<resident_grid<K, 64>(cfg.ncu, cfg.wgs_s), 64, 0, st>>>(
            w.sent, w.nactive, b->src_idx, g, w.s, w.G, w.rmask, w.tmask, use_dv);
    }
}

// The tile spreading, with or without the slot row masks.
template <typename T, int P>
static void launch_spread(const BatchedCfg& cfg, hipStream_t st, const Grid& g,
                          const BatchedWs<T>& w, const ib_buckets* b, int use_dv)
{
    if (cfg.masks)
        spread_kernel<T, P, true>(cfg, st, g, w, b, use_dv);
    else
        spread_kernel<T, P, false>(cfg, st, g, w, b, use_dv);
}

#define IBX_PROF_BEGIN(k) \
    if (cfg.prof) cfg.prof->begin(k, st)
#define IBX_PROF_END() \
    if (cfg.prof) cfg.prof->end(st)

// Work lists of the interpolation items (work tiles of one tile, or with
// PAIR of two x neighbours) and of the active tiles, and each item's
// neighbour offsets.
// The list pass that k_prep_lists runs beside the records: the fused list
// scan for grids of at most SCAN_FUSE / 2 scan tiles, else the tile counts.
static bool fused_list_scan(const Grid& g)
{
    return 2 * ((g.ntiles + SCAN_TILE - 1) / SCAN_TILE) <= SCAN_FUSE;
}

// The rest of the work lists, after k_prep_lists.
template <typename T, bool PAIR>
static void build_lists(const Grid& g, const BatchedCfg& cfg, const ib_buckets* b,
                        BatchedWs<T>& w, hipStream_t st)
{
    const int64_t T_ = g.ntiles;
    const unsigned gt = (unsigned)((T_ + 255) / 256);
    const int64_t nbl = (T_ + SCAN_TILE - 1) / SCAN_TILE;
    if (fused_list_scan(g)) {
        int32_t* sums = (int32_t*)w.scan;
        k_list_add<PAIR><<<(unsigned)(2 * nbl), SCAN_THREADS, 0, st>>>(
            T_, b->src_offs, w.item_offs, w.act_offs, sums, w.nitems, w.nactive, w.hist, cfg.bw,
            g.nt[0], b->tile_offs, w.items);
    } else {
        scan_exclusive2(w.item_cnt, w.item_offs, w.act, w.act_offs, T_, w.nitems, w.nactive,
                        w.scan, st);
        k_cost_hist<PAIR><<<gt, 256, 0, st>>>(T_, b->src_offs, w.act_offs, w.nactive, w.hist,
                                              cfg.bw, g.nt[0], b->tile_offs, w.item_offs,
                                              w.items);
    }
    constexpr int NBX = PAIR ? 4 : 3;
    const int64_t nth = 9 * NBX * w.max_items;
    k_bins_bases<PAIR><<<(unsigned)(NXCD + (nth + COST_BINS - 1) / COST_BINS), COST_BINS, 0, st>>>(
        w.hist, w.nactive, w.cur, g, w.items, w.nitems, b->src_offs, w.act_offs, w.nb_u, w.nb_g);
    k_fill_lists<<<gt, 256, 0, st>>>(T_, b->src_offs, w.act_offs, w.nactive, w.slot, w.cur,
                                     w.sent);
}

// Marker records in bucket order and the work lists of the tile kernels
// (interpolation items, G slots, spreading order, neighbour offsets).
template <typename T, int P>
static void records_and_lists(const Grid& g, const BatchedCfg& cfg, const ib_particles* p,
                              const ib_markers* m, const ib_buckets* b, BatchedWs<T>& w,
                              hipStream_t st)
{
    const int64_t nl = m->nl;
    const unsigned gm = (unsigned)((nl + 255) / 256);
    const bool scan = fused_list_scan(g);
    const unsigned nlist = (unsigned)(scan ? 2 * ((g.ntiles + SCAN_TILE - 1) / SCAN_TILE)
                                           : (g.ntiles + 255) / 256);
    int32_t* out_items = scan ? w.item_offs : w.item_cnt;
    int32_t* out_act = scan ? w.act_offs : w.act;
    const bool pair = pair_items<T>(cfg);
    IBX_PROF_BEGIN(PK_PREP);
#define IBX_PREP_LISTS(PAIR, SCAN)                                                               \
    k_prep_lists<T, P, PAIR, SCAN><<<nlist + gm, 256, 0, st>>>(                                  \
        nlist, g, nl, m->x, m->y, m->z, m->pid, m->dv, b->perm, p->xc, p->up, p->om, w.s, cfg.bw, \
        b->tile_offs, b->src_offs, out_items, out_act, (int32_t*)w.scan, w.hist)
    if (pair && scan)
        IBX_PREP_LISTS(true, true);
    else if (pair)
        IBX_PREP_LISTS(true, false);
    else if (scan)
        IBX_PREP_LISTS(false, true);
    else
        IBX_PREP_LISTS(false, false);
#undef IBX_PREP_LISTS
    IBX_PROF_END();
    IBX_PROF_BEGIN(PK_LISTS);
    if (pair)
        build_lists<T, true>(g, cfg, b, w, st);
    else
        build_lists<T, false>(g, cfg, b, w, st);
    IBX_PROF_END();
}

// Every output set to NaN when the bucket set is flagged (checked on the
// device at the end of the loop; nothing is read back).
template <typename T>
static void poison_outputs(const Grid& g, const ib_buckets* b, T* ustar, T* f, T* F,
                           double* resid, T* Fhist, int64_t nl, int ns, hipStream_t st)
{
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
}

template <typename T, int P>
static int run_batched(const Grid& g, const BatchedCfg& cfg, const ib_particles* p,
                       const ib_markers* m, const ib_buckets* b, int ns, double dt,
                       const T* u0, T* ustar, T* f, T* F, double* resid, T* Fhist, void* ws,
                       size_t ws_bytes, hipStream_t st, int f_acc)
{
    const int64_t nl = m->nl;
    size_t need = 0;
    carve_batched<T>(g, nl, cfg.bw, nullptr, 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    BatchedWs<T> w = carve_batched<T>(g, nl, cfg.bw, ws, ws_bytes, &need);
    const unsigned gm = (unsigned)((nl + 255) / 256 > 0 ? (nl + 255) / 256 : 1);
    const int64_t nfin = (int64_t)g.nbox * (g.box / TILE) * g.box;
    const unsigned gfin = (unsigned)(nfin < 65535 ? (nfin > 0 ? nfin : 1) : 65535);
    if (nl == 0) {
        launch_finalize<T>(gfin, st, g, w.slot, w.G, w.tmask, u0, ustar, f, dt, 0, f_acc,
                          cfg.masks);
        if (resid)
            k_zero<double><<<1, 64, 0, st>>>(ns + 1, resid);
        poison_outputs(g, b, ustar, f, F, resid, Fhist, nl, ns, st);
        return launch_status();
    }
    records_and_lists<T, P>(g, cfg, p, m, b, w, st);
    double* e2 = resid ? w.e2 : nullptr;
    IBX_PROF_BEGIN(PK_INTERP_U0);
    // the last interpolation of the loop also writes F in marker order
    launch_interp<T, P, 0>(cfg, st, g, nl, dt, w.items, w.nitems, u0, w.G, w.rmask, w.nb_u, w.s,
                           e2, ns == 1 ? F : nullptr, b->perm);
    IBX_PROF_END();
    if (resid)
        sum_to(w.e2, nl, w.part, resid + 0, true, st);
    if (ns == 0) {
        // no iteration: ustar = u0, f = 0, F = 0
        launch_finalize<T>(gfin, st, g, w.slot, w.G, w.tmask, u0, ustar, f, dt, 0, f_acc,
                          cfg.masks);
        k_zero<T><<<gm, 256, 0, st>>>(3 * nl, F);
        poison_outputs(g, b, ustar, f, F, resid, Fhist, nl, ns, st);
        return launch_status();
    }
    if (Fhist)
        k_unsort<T><<<gm, 256, 0, st>>>(nl, b->perm, w.s.f4, Fhist);
    for (int mi = 2; mi <= ns; ++mi) {
        IBX_PROF_BEGIN(PK_SPREAD);
        launch_spread<T, P>(cfg, st, g, w, b, 1);
        IBX_PROF_END();
        IBX_PROF_BEGIN(PK_INTERP_G);
        launch_interp<T, P, 1>(cfg, st, g, nl, dt, w.items, w.nitems, u0, w.G, w.rmask, w.nb_g,
                               w.s, e2, mi == ns ? F : nullptr, b->perm);
        IBX_PROF_END();
        if (resid)
            sum_to(w.e2, nl, w.part, resid + (mi - 1), true, st);
        if (Fhist)
            k_unsort<T><<<gm, 256, 0, st>>>(nl, b->perm, w.s.f4,
                                            Fhist + (int64_t)(mi - 1) * 3 * nl);
    }
    IBX_PROF_BEGIN(PK_SPREAD_FINAL);
    launch_spread<T, P>(cfg, st, g, w, b, 1);
    IBX_PROF_END();
    // without residuals or force history, the finalize writes the last
    // outputs (F is written before it) and checks the flags itself
    const bool fold = !resid && !Fhist;
    IBX_PROF_BEGIN(PK_FILL);
    launch_finalize<T>(gfin, st, g, w.slot, w.G, w.tmask, u0, ustar, f, dt, 1, f_acc, cfg.masks,
                       fold ? b->flag : nullptr, F, 3 * nl);
    IBX_PROF_END();
    if (resid) {
        IBX_PROF_BEGIN(PK_RESID);
        launch_interp<T, P, 2>(cfg, st, g, nl, dt, w.items, w.nitems, u0, w.G, w.rmask, w.nb_g,
                               w.s, w.e2);
        IBX_PROF_END();
        sum_to(w.e2, nl, w.part, resid + ns, true, st);
    }
    if (!fold)
        poison_outputs(g, b, ustar, f, F, resid, Fhist, nl, ns, st);
    return launch_status();
}

// ------------------------------------------------------------------ spreading outside the loop

// The spreads of the adjoint (the recomputed u^(m-1) = u0 + dt S F^(m-1) and
// the transpose of interpolation, J^T Ubar) run on the loop's tile kernel:
// tile_spread_setup forms the marker records and work lists once per call,
// then each tile_spread puts its marker vector into bucket order, spreads it
// into the G slots and writes the field.

template <typename T>
__global__ void k_sort_vec(int64_t nl, const int32_t* __restrict__ perm, const T* __restrict__ v,
                           typename Vec4<T>::type* __restrict__ f4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl)
        return;
    const int64_t l = perm[i];
    typename Vec4<T>::type q;
    q.x = v[3 * l];
    q.y = v[3 * l + 1];
    q.z = v[3 * l + 2];
    q.w = T(0);
    f4[i] = q;
}

bool tile_spread_supported(const Grid& g)
{
    for (int a = 0; a < 3; ++a)
        if (g.n[a] < 2 * TILE || g.n[a] > (int)RB_MASK - RB_BIAS)
            return false;
    return g.box <= 64 * TILE;
}

size_t tile_spread_workspace(const Grid& g, ib_prec prec, int64_t nl)
{
    BatchedCfg c{};
    c.bw = 64;
    return batched_workspace(g, prec, nl, c);
}

template <typename T, int P>
static void setup_t(const Grid& g, const BatchedCfg& cfg, const ib_particles* p,
                    const ib_markers* m, const ib_buckets* b, void* ws, size_t bytes,
                    hipStream_t st)
{
    size_t need = 0;
    BatchedWs<T> w = carve_batched<T>(g, m->nl, cfg.bw, ws, bytes, &need);
    records_and_lists<T, P>(g, cfg, p, m, b, w, st);
}

int tile_spread_setup(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                      const ib_particles* p, const ib_markers* m, const ib_buckets* b, void* ws,
                      size_t ws_bytes, hipStream_t st)
{
    if (ws_bytes < tile_spread_workspace(g, prec, m->nl) || m->nl == 0)
        return m->nl == 0 ? IB_OK : IB_EWORKSPACE;
    BatchedCfg c = cfg;
    c.prof = nullptr;
    if (prec == IB_F64)
        P == 3 ? setup_t<double, 3>(g, c, p, m, b, ws, ws_bytes, st)
               : setup_t<double, 4>(g, c, p, m, b, ws, ws_bytes, st);
    else
        P == 3 ? setup_t<float, 3>(g, c, p, m, b, ws, ws_bytes, st)
               : setup_t<float, 4>(g, c, p, m, b, ws, ws_bytes, st);
    return launch_status();
}

template <typename T, int P>
static void spread_t(const Grid& g, const BatchedCfg& cfg, const ib_markers* m,
                     const ib_buckets* b, const T* v, int use_dv, const T* u0, double dt, T* out,
                     void* ws, size_t bytes, hipStream_t st)
{
    size_t need = 0;
    const int64_t nl = m->nl;
    BatchedWs<T> w = carve_batched<T>(g, nl, cfg.bw, ws, bytes, &need);
    const int64_t nfin = (int64_t)g.nbox * (g.box / TILE) * g.box;
    const unsigned gfin = (unsigned)(nfin < 65535 ? (nfin > 0 ? nfin : 1) : 65535);
    if (nl > 0) {
        k_sort_vec<T><<<(unsigned)((nl + 255) / 256), 256, 0, st>>>(nl, b->perm, v, w.s.f4);
        launch_spread<T, P>(cfg, st, g, w, b, use_dv);
    }
    // u0 given: out = u0 + dt G; else out = G (zero where no marker reaches)
    if (u0)
        launch_finalize<T>(gfin, st, g, w.slot, w.G, w.tmask, u0, out, nullptr, dt, nl > 0, 0,
                          cfg.masks);
    else
        launch_finalize<T>(gfin, st, g, w.slot, w.G, w.tmask, nullptr, nullptr, out, dt, nl > 0, 0,
                          cfg.masks);
}

int tile_spread(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg, const ib_markers* m,
                const ib_buckets* b, const void* v, int use_dv, const void* u0, double dt,
                void* out, void* ws, size_t ws_bytes, hipStream_t st)
{
    if (ws_bytes < tile_spread_workspace(g, prec, m->nl))
        return IB_EWORKSPACE;
    if (prec == IB_F64) {
        if (P == 3)
            spread_t<double, 3>(g, cfg, m, b, (const double*)v, use_dv, (const double*)u0, dt,
                                (double*)out, ws, ws_bytes, st);
        else
            spread_t<double, 4>(g, cfg, m, b, (const double*)v, use_dv, (const double*)u0, dt,
                                (double*)out, ws, ws_bytes, st);
    } else {
        if (P == 3)
            spread_t<float, 3>(g, cfg, m, b, (const float*)v, use_dv, (const float*)u0, dt,
                               (float*)out, ws, ws_bytes, st);
        else
            spread_t<float, 4>(g, cfg, m, b, (const float*)v, use_dv, (const float*)u0, dt,
                               (float*)out, ws, ws_bytes, st);
    }
    return launch_status();
}

template <typename T, int P>
static void interp_grad_t(const Grid& g, const BatchedCfg& cfg, const ib_markers* m,
                          const ib_buckets* b, const T* fld, const T* v, T* U, int use_dv,
                          double* gX, void* ws, size_t bytes, hipStream_t st)
{
    size_t need = 0;
    BatchedWs<T> w = carve_batched<T>(g, m->nl, cfg.bw, ws, bytes, &need);
    launch_interp<T, P, 3>(cfg, st, g, m->nl, 0.0, w.items, w.nitems, fld, nullptr, nullptr,
                           w.nb_u, w.s, nullptr, U, b->perm, v, gX, use_dv);
}

int tile_interp_grad(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                     const ib_markers* m, const ib_buckets* b, const void* fld, const void* v,
                     void* U, int use_dv, double* gX, void* ws, size_t ws_bytes, hipStream_t st)
{
    if (ws_bytes < tile_spread_workspace(g, prec, m->nl))
        return IB_EWORKSPACE;
    if (m->nl == 0)
        return IB_OK;
    if (prec == IB_F64) {
        if (P == 3)
            interp_grad_t<double, 3>(g, cfg, m, b, (const double*)fld, (const double*)v,
                                     (double*)U, use_dv, gX, ws, ws_bytes, st);
        else
            interp_grad_t<double, 4>(g, cfg, m, b, (const double*)fld, (const double*)v,
                                     (double*)U, use_dv, gX, ws, ws_bytes, st);
    } else {
        if (P == 3)
            interp_grad_t<float, 3>(g, cfg, m, b, (const float*)fld, (const float*)v,
                                    (float*)U, use_dv, gX, ws, ws_bytes, st);
        else
            interp_grad_t<float, 4>(g, cfg, m, b, (const float*)fld, (const float*)v,
                                    (float*)U, use_dv, gX, ws, ws_bytes, st);
    }
    return launch_status();
}

size_t batched_workspace(const Grid& g, ib_prec prec, int64_t nl, const BatchedCfg& cfg)
{
    size_t need = 0;
    if (prec == IB_F64)
        carve_batched<double>(g, nl, cfg.bw, nullptr, 0, &need);
    else
        carve_batched<float>(g, nl, cfg.bw, nullptr, 0, &need);
    return need;
}

int batched_multidirect(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                        const ib_particles* p, const ib_markers* m, const ib_buckets* b, int ns,
                        double dt, const void* u0, void* ustar, void* f, void* F, double* resid,
                        void* Fhist, void* ws, size_t ws_bytes, hipStream_t st, int f_acc)
{
    // a stencil must never reach the same tile from both sides of a periodic
    // axis; every stencil base (>= -2, < n) fits a packed field
    for (int a = 0; a < 3; ++a)
        if (g.n[a] < 2 * TILE || g.n[a] > (int)RB_MASK - RB_BIAS)
            return IB_EUNSUPPORTED;
    // the finalize step holds one box row of tile slots in LDS
    if (g.box > 64 * TILE)
        return IB_EUNSUPPORTED;
    if (prec == IB_F64) {
        if (P == 3)
            return run_batched<double, 3>(g, cfg, p, m, b, ns, dt, (const double*)u0,
                                          (double*)ustar, (double*)f, (double*)F, resid,
                                          (double*)Fhist, ws, ws_bytes, st, f_acc);
        return run_batched<double, 4>(g, cfg, p, m, b, ns, dt, (const double*)u0,
                                      (double*)ustar, (double*)f, (double*)F, resid,
                                      (double*)Fhist, ws, ws_bytes, st, f_acc);
    }
    if (P == 3)
        return run_batched<float, 3>(g, cfg, p, m, b, ns, dt, (const float*)u0, (float*)ustar,
                                     (float*)f, (float*)F, resid, (float*)Fhist, ws, ws_bytes,
                                     st, f_acc);
    return run_batched<float, 4>(g, cfg, p, m, b, ns, dt, (const float*)u0, (float*)ustar,
                                 (float*)f, (float*)F, resid, (float*)Fhist, ws, ws_bytes, st,
                                 f_acc);
}

}  // namespace ibx
