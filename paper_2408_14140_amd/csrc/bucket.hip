// bucket.hip -- a2: markers bucketed by owning 8^3 tile, and per-tile source
// lists.  Integer work only; every output is deterministic.
//
// Pipeline (all on one stream, no host synchronization):
//   keys    per marker: owning cell, tile, stencil base, coverage check, and
//           the directions of the tiles its stencil touches
//   sort    stable LSD radix sort of (tile, marker) -> perm
//   offs    tile_offs[t] = lower bound of t in the sorted tiles
//   lists   src_idx / src_offs (each list ascending in the sorted position):
//           with 3 or more tiles on every axis, by direction (per owning
//           tile, runs counted and written with ballots, placed by one scan);
//           otherwise the (tile, i) pairs of every touched tile, emitted in
//           i order and stably sorted by tile
#include "ibx_internal.h"

namespace ibx {

// ------------------------------------------------------------------ scan

// total (if not null) receives the sum of the whole input: launch it only
// with one workgroup then.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tile(const int32_t* in, int32_t* out, int64_t n, int32_t* sums, int shift,
            int32_t* total)
{
    __shared__ int32_t ts[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? (in[base + k] >> shift) : 0;
        tsum += v[k];
    }
    ts[t] = tsum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int32_t x = (t >= off) ? ts[t - off] : 0;
        __syncthreads();
        ts[t] += x;
        __syncthreads();
    }
    int32_t run = ts[t] - tsum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n)
            out[base + k] = run;
        run += v[k];
    }
    if (t == SCAN_THREADS - 1) {
        sums[blockIdx.x] = ts[t];
        if (total)
            *total = ts[t];
    }
}

// sums: the scanned tile totals, or (fused) the tile totals themselves, whose
// prefix each workgroup forms; the last workgroup then writes the total.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_add(int32_t* out, int64_t n, const int32_t* sums, bool fused, int32_t* total)
{
    const int32_t add = fused ? group_sum(sums, blockIdx.x) : sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += blockDim.x)
        if (base + k < n)
            out[base + k] += add;
    if (fused && total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1)
        *total = add + sums[blockIdx.x];
}

__global__ void k_set1(int32_t* dst, int32_t v) { *dst = v; }

size_t scan_workspace(int64_t n)
{
    size_t bytes = 0;
    while (n > 0) {
        int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        bytes += align_up(sizeof(int32_t) * nb);
        if (nb == 1)
            break;
        n = nb;
    }
    return bytes + 256;
}

void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* ws,
                    hipStream_t st, int shift)
{
    if (n <= 0) {
        if (total)
            k_set1<<<1, 1, 0, st>>>(total, 0);
        return;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* sums = (int32_t*)ws;
    k_scan_tile<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(in, out, n, sums, shift,
                                                       nb == 1 ? total : nullptr);
    if (nb == 1)
        return;
    if (nb <= SCAN_FUSE) {
        k_scan_add<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(out, n, sums, true, total);
        return;
    }
    scan_exclusive(sums, sums, nb, total, (char*)ws + align_up(sizeof(int32_t) * nb), st, 0);
    k_scan_add<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(out, n, sums, false, nullptr);
}

// Two independent scans of the same length in one pass per level: block b
// of the first kernel scans tile b of array 0 (b < nb) or tile b - nb of
// array 1.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tile2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1, int64_t n,
             int32_t* sums)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    const bool second = blockIdx.x >= nb;
    const int64_t blk = second ? blockIdx.x - nb : blockIdx.x;
    const int32_t* in = second ? in1 : in0;
    int32_t* out = second ? out1 : out0;
    __shared__ int32_t ts[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t base = blk * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        tsum += v[k];
    }
    ts[t] = tsum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int32_t x = (t >= off) ? ts[t - off] : 0;
        __syncthreads();
        ts[t] += x;
        __syncthreads();
    }
    int32_t run = ts[t] - tsum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n)
            out[base + k] = run;
        run += v[k];
    }
    if (t == SCAN_THREADS - 1)
        sums[blockIdx.x] = ts[t];
}

// Adds the scanned tile sums back (sums holds both arrays' tiles, nb each);
// blocks 2 nb and 2 nb + 1 ... are not used: the totals come from the last
// tile of each array.  With sums_scan null, each workgroup forms the prefix
// of the tile totals itself.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_add2(int32_t* out0, int32_t* out1, int64_t n, const int32_t* sums_scan,
            const int32_t* sums, int32_t* total0, int32_t* total1)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    const bool second = blockIdx.x >= nb;
    const int64_t blk = second ? blockIdx.x - nb : blockIdx.x;
    int32_t* out = second ? out1 : out0;
    // exclusive prefix of this array's tiles = scan of all tiles minus the
    // first array's total for the second array
    const int32_t pre = sums_scan ? sums_scan[blockIdx.x] : group_sum(sums, blockIdx.x);
    const int32_t first_total = sums_scan ? sums_scan[nb - 1] + sums[nb - 1] : group_sum(sums, nb);
    const int32_t add = pre - (second ? first_total : 0);
    const int64_t base = blk * SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += blockDim.x)
        if (base + k < n)
            out[base + k] += add;
    if (threadIdx.x == 0 && blk == nb - 1) {
        const int32_t tot = pre + sums[blockIdx.x] - (second ? first_total : 0);
        if (second) {
            if (total1)
                *total1 = tot;
        } else if (total0) {
            *total0 = tot;
        }
    }
}

size_t scan2_workspace(int64_t n)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return 2 * align_up(sizeof(int32_t) * 2 * (nb > 0 ? nb : 1)) + scan_workspace(2 * nb);
}

void scan_exclusive2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1,
                     int64_t n, int32_t* total0, int32_t* total1, void* ws, hipStream_t st)
{
    if (n <= 0) {
        if (total0)
            k_set1<<<1, 1, 0, st>>>(total0, 0);
        if (total1)
            k_set1<<<1, 1, 0, st>>>(total1, 0);
        return;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* sums = (int32_t*)ws;
    int32_t* sscan = (int32_t*)((char*)ws + align_up(sizeof(int32_t) * 2 * nb));
    void* rest = (char*)ws + 2 * align_up(sizeof(int32_t) * 2 * nb);
    k_scan_tile2<<<(unsigned)(2 * nb), SCAN_THREADS, 0, st>>>(in0, out0, in1, out1, n, sums);
    const bool fused = 2 * nb <= SCAN_FUSE;
    if (!fused)
        scan_exclusive(sums, sscan, 2 * nb, nullptr, rest, st, 0);
    k_scan_add2<<<(unsigned)(2 * nb), SCAN_THREADS, 0, st>>>(out0, out1, n,
                                                             fused ? nullptr : sscan, sums,
                                                             total0, total1);
}

// ------------------------------------------------------------------ radix sort

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / 64;

__device__ inline int64_t live_count(int64_t n_max, const int32_t* n_dev)
{
    if (!n_dev)
        return n_max;
    int64_t v = *n_dev;
    return v < n_max ? v : n_max;
}

__global__ void __launch_bounds__(RS_THREADS)
k_radix_hist(const int32_t* keys, int64_t n_max, const int32_t* n_dev, int shift,
             int32_t* hist, int nblocks)
{
    __shared__ int32_t h[256];
    const int t = threadIdx.x;
    const int64_t n = live_count(n_max, n_dev);
    h[t] = 0;
    __syncthreads();
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t j = (int64_t)blockIdx.x * RS_TILE + r * RS_THREADS + t;
        if (j < n)
            atomicAdd(&h[(keys[j] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Exclusive scan of one digit's row of block counts (workgroup d scans
// hist[d][0 .. nblocks)); rowtot[d] receives the row's total.
__global__ void __launch_bounds__(RS_THREADS)
k_radix_rowscan(int32_t* hist, int nblocks, int32_t* rowtot)
{
    __shared__ int32_t ts[RS_THREADS];
    const int t = threadIdx.x;
    int32_t* row = hist + (int64_t)blockIdx.x * nblocks;
    int32_t carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += RS_THREADS * 4) {
        int32_t v[4];
        int32_t tsum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = c0 + 4 * t + k;
            v[k] = j < nblocks ? row[j] : 0;
            tsum += v[k];
        }
        ts[t] = tsum;
        __syncthreads();
        for (int off = 1; off < RS_THREADS; off <<= 1) {
            const int32_t x = t >= off ? ts[t - off] : 0;
            __syncthreads();
            ts[t] += x;
            __syncthreads();
        }
        int32_t run = carry + ts[t] - tsum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = c0 + 4 * t + k;
            if (j < nblocks)
                row[j] = run;
            run += v[k];
        }
        carry += ts[RS_THREADS - 1];
        __syncthreads();
    }
    if (t == 0)
        rowtot[blockIdx.x] = carry;
}

// Stable scatter: elements keep their input order within each digit.  Ranks
// inside a wave come from ballot matching on the 8 digit bits; ranks across
// the block's waves and rounds from per-digit counters in LDS.
__global__ void __launch_bounds__(RS_THREADS)
k_radix_scatter(const int32_t* kin, const int32_t* vin, int32_t* kout, int32_t* vout,
                int64_t n_max, const int32_t* n_dev, int shift, const int32_t* hist_scan,
                const int32_t* rowtot, int nblocks)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wc[RS_WAVES][256];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int64_t n = live_count(n_max, n_dev);
    if ((int64_t)blockIdx.x * RS_TILE >= n)
        return;                             // whole block past the live count
    // digit offsets: exclusive scan of the digit totals, in every block
    const int32_t tot = rowtot[t];
    run[t] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t xv = t >= off ? run[t - off] : 0;
        __syncthreads();
        run[t] += xv;
        __syncthreads();
    }
    const int32_t doff = run[t] - tot;
    __syncthreads();
    run[t] = doff + hist_scan[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w)
        wc[w][t] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t j = (int64_t)blockIdx.x * RS_TILE + r * RS_THREADS + t;
        const bool valid = j < n;
        const int32_t k = valid ? kin[j] : 0;
        const int32_t v = valid ? vin[j] : 0;
        const int d = (k >> shift) & 255;
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(valid && bit);
            mask &= bit ? m : ~m;
        }
        const int rank = __popcll(mask & lt);
        if (valid && rank == 0)
            wc[wave][d] = __popcll(mask);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w)
                pos += wc[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            add += wc[w][t];
            wc[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

__global__ void k_copy_pairs(const int32_t* ks, const int32_t* vs, int32_t* kd, int32_t* vd,
                             int64_t n_max, const int32_t* n_dev)
{
    const int64_t n = live_count(n_max, n_dev);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        kd[j] = ks[j];
        vd[j] = vs[j];
    }
}

static int64_t rs_blocks(int64_t n_max) { return (n_max + RS_TILE - 1) / RS_TILE; }

size_t radix_workspace(int64_t n_max)
{
    int64_t nb = rs_blocks(n_max > 0 ? n_max : 1);
    return align_up(sizeof(int32_t) * 256 * nb) + align_up(sizeof(int32_t) * 256);
}

void radix_sort_pairs(int32_t* keys, int32_t* vals, int32_t* tk, int32_t* tv, int64_t n_max,
                      const int32_t* n_dev, int bits, void* ws, hipStream_t st)
{
    if (n_max <= 0 || bits <= 0)
        return;
    const int64_t nb = rs_blocks(n_max);
    int32_t* hist = (int32_t*)ws;
    int32_t* rowtot = (int32_t*)((char*)ws + align_up(sizeof(int32_t) * 256 * nb));
    int32_t *ka = keys, *va = vals, *kb = tk, *vb = tv;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_radix_hist<<<(unsigned)nb, RS_THREADS, 0, st>>>(ka, n_max, n_dev, shift, hist, (int)nb);
        k_radix_rowscan<<<256, RS_THREADS, 0, st>>>(hist, (int)nb, rowtot);
        k_radix_scatter<<<(unsigned)nb, RS_THREADS, 0, st>>>(ka, va, kb, vb, n_max, n_dev, shift,
                                                             hist, rowtot, (int)nb);
        int32_t* t0 = ka; ka = kb; kb = t0;
        t0 = va; va = vb; vb = t0;
    }
    if (ka != keys) {
        int64_t g = (n_max + 255) / 256;
        if (g > 65536)
            g = 65536;
        k_copy_pairs<<<(unsigned)g, 256, 0, st>>>(ka, va, keys, vals, n_max, n_dev);
    }
}

__global__ void k_lower_bounds(const int32_t* keys, int64_t n_max, const int32_t* n_dev,
                               int32_t* offs, int64_t T, int32_t mask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T)
        return;
    int64_t lo = 0, hi = live_count(n_max, n_dev);
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] & mask) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    offs[t] = (int32_t)lo;
}

void lower_bounds(const int32_t* keys, int64_t n_max, const int32_t* n_dev, int32_t* offs,
                  int64_t T, hipStream_t st, int32_t mask)
{
    k_lower_bounds<<<(unsigned)((T + 1 + 255) / 256), 256, 0, st>>>(keys, n_max, n_dev, offs, T,
                                                                    mask);
}

// ------------------------------------------------------------------ bucket keys

// Clears the two flags and a[0 .. n).
__global__ void k_init_flags(int32_t* flag, int64_t n, int32_t* __restrict__ a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2)
        flag[i] = 0;
    if (i < n)
        a[i] = 0;
}

// Tiles touched on one axis by the stencil cells b .. b+P-1 (1 or 2 tiles).
template <int P>
__device__ inline int axis_tiles(const Grid& g, int a, int b, int* tl)
{
    int nt = 0;
    for (int o = 0; o < P; ++o) {
        int q = b + o;
        if (g.periodic[a])
            q = wrapi(q, g.n[a]);
        else if (q < 0 || q >= g.n[a])
            continue;
        const int tq = q / TILE;
        if (nt == 0 || (tl[nt - 1] != tq && nt < 2 && tl[0] != tq))
            tl[nt++] = tq;
    }
    return nt;
}

// Source lists by direction.  With at least 3 tiles on every axis the 27
// tiles around an owning tile are distinct.  The source list of tile t is
// then the concatenation, over its 27 neighbours t' in increasing index
// order, of the markers owned by t' whose stencil touches t, each run in
// sorted-position order: the same ascending list that a stable sort of the
// (tile, position) pairs gives.  Each marker's directions are found with its
// key, each owning tile counts its markers per direction, the runs are
// placed by one scan over the tiles, and each owning tile writes its runs
// with ballot ranks.
constexpr int NDIR = 27;

__device__ inline void tile_xyz(const Grid& g, int64_t t, int* c)
{
    const int ti = (int)t;          // tile indices fit 31 bits (cells do)
    c[0] = ti % g.nt[0];
    c[1] = (ti / g.nt[0]) % g.nt[1];
    c[2] = ti / (g.nt[0] * g.nt[1]);
}

// The tile at tc + s (d): s = +1 gives the tile that a run from tc in
// direction d reaches, s = -1 the owner of the run that tc receives from
// direction d.  -1 past a bounded edge.
__device__ inline int64_t dir_tile(const Grid& g, const int* tc, int d, int s)
{
    const int dd[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
    int oc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = tc[a] + s * dd[a];
        if (v < 0 || v >= g.nt[a]) {
            if (!g.periodic[a])
                return -1;
            v = v < 0 ? v + g.nt[a] : v - g.nt[a];
        }
        oc[a] = v;
    }
    return oc[0] + (int64_t)g.nt[0] * (oc[1] + (int64_t)g.nt[1] * oc[2]);
}

// The 27-bit direction set (bit (dx + 1) + 3 (dy + 1) + 9 (dz + 1)) of a
// direction code.
__device__ inline uint32_t dir_set(int code)
{
    uint32_t ax[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int k = (code >> (2 * a)) & 3;
        ax[a] = k == 1 ? 3u : k == 2 ? 6u : 2u;     // {-1, 0}, {0, +1}, {0}
    }
    uint32_t r = 0;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                if ((ax[2] >> dz) & (ax[1] >> dy) & (ax[0] >> dx) & 1)
                    r |= 1u << (dx + 3 * dy + 9 * dz);
    return r;
}

// Per marker: owning cell c = floor(s) (wrapped on periodic axes), its tile,
// the unwrapped stencil base, and whether all stencil cells are covered.  The
// sort key is the tile; with kb > 0 the number of tiles the stencil touches
// rides above the sorted digits, at bit kb.  dmask (nullable) receives the
// directions of the touched tiles from the owning one (dir_set of the
// direction code: per axis the owning tile's layer alone, with the layer
// below, or with the layer above -- the owning cell is always in the stencil,
// and with 3 or more tiles on the axis the P cells reach one neighbour layer
// at most).  Without dmask a marker whose stencil leaves the coverage adds 1
// to flag[0]; with it, such a marker sets bit 31 of its dmask entry (for
// k_dir_counts to count), and this kernel clears the two flags and
// ztot[0 .. nz) first (nothing raises them before k_dir_counts).
template <int P>
__global__ void k_bucket_keys(Grid g, int64_t nl, const double* __restrict__ x,
                              const double* __restrict__ y, const double* __restrict__ z,
                              int32_t* cell, int32_t* tileid, int32_t* base, int32_t* keys,
                              int32_t* vals, int32_t* flag, int kb, uint32_t* dmask, int64_t nz,
                              int32_t* __restrict__ ztot)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (dmask) {
        if (l < 2)
            flag[l] = 0;
        for (int64_t i = l; i < nz; i += (int64_t)gridDim.x * blockDim.x)
            ztot[i] = 0;
    }
    if (l >= nl)
        return;
    const double X[3] = {x[l], y[l], z[l]};
    int c[3], b[3];
    int bad = 0, tcount = 1;
    int bx[3][2], nbx[3];
    int code = 0;                   // direction code, 2 bits per axis
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = grid_coord(g, a, X[a]);
        const int fl = (int)floor(s);
        b[a] = stencil_base<P>(s);
        // first and last stencil cell on this axis (wrapped, or clipped to a
        // bounded axis): the P consecutive cells lie in at most two boxes and
        // two tiles, those of these two cells
        int q0, q1;
        if (g.periodic[a]) {
            // markers sit at most a period outside: one add or subtract, else
            // the modulo
            c[a] = fl < 0 ? fl + g.n[a] : fl >= g.n[a] ? fl - g.n[a] : fl;
            if ((unsigned)c[a] >= (unsigned)g.n[a])
                c[a] = wrapi(fl, g.n[a]);
            q0 = b[a] < 0 ? b[a] + g.n[a] : b[a] >= g.n[a] ? b[a] - g.n[a] : b[a];
            if ((unsigned)q0 >= (unsigned)g.n[a])
                q0 = wrapi(b[a], g.n[a]);
            q1 = q0 + P - 1;
            if (q1 >= g.n[a])
                q1 -= g.n[a];
        } else {
            c[a] = fl;
            if (fl < 0 || fl >= g.n[a]) {
                bad = 1;
                c[a] = fl < 0 ? 0 : g.n[a] - 1;
            }
            q0 = max(b[a], 0);
            q1 = min(b[a] + P - 1, g.n[a] - 1);
            if (b[a] < 0 || b[a] + P - 1 >= g.n[a])
                bad = 1;
        }
        if (g.periodic[a] || q0 <= q1) {
            bx[a][0] = q0 / g.box;
            bx[a][1] = q1 / g.box;
            nbx[a] = bx[a][1] != bx[a][0] ? 2 : 1;
            tcount *= (q1 >> 3) != (q0 >> 3) ? 2 : 1;
            // the P cells span at most two tiles, those of q0 and q1
            const int ot = c[a] / TILE;
            if ((q0 >> 3) != ot)
                code |= 1 << (2 * a);
            else if ((q1 >> 3) != ot)
                code |= 2 << (2 * a);
        } else {
            nbx[a] = 0;
            tcount = 0;
        }
    }
    for (int k = 0; k < nbx[2] && !bad; ++k)
        for (int j = 0; j < nbx[1] && !bad; ++j)
            for (int i = 0; i < nbx[0] && !bad; ++i)
                if (g.lut[bx[0][i] + g.nb[0] * (bx[1][j] + g.nb[1] * bx[2][k])] < 0)
                    bad = 1;
    cell[l] = c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
    const int t = c[0] / TILE + g.nt[0] * (c[1] / TILE + g.nt[1] * (c[2] / TILE));
    tileid[l] = t;
    int key = t;
    if (kb > 0)
        key |= tcount << kb;
    if (dmask)
        dmask[l] = dir_set(code) | (bad ? 1u << 31 : 0u);
    keys[l] = key;
    vals[l] = (int32_t)l;
    base[3 * l + 0] = b[0];
    base[3 * l + 1] = b[1];
    base[3 * l + 2] = b[2];
    if (bad && !dmask)
        atomicAdd(&flag[0], 1);
}

template <int P>
__global__ void k_src_count(Grid g, int64_t nl, const int32_t* perm, const int32_t* base,
                            int32_t* cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl)
        return;
    const int64_t l = perm[i];
    int tl[2], c = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        c *= axis_tiles<P>(g, a, base[3 * l + a], tl);
    cnt[i] = c;
}

// npairs[0] = min(total pairs, cap), written by the last marker.
template <int P>
__global__ void k_src_emit(Grid g, int64_t nl, const int32_t* perm, const int32_t* base,
                           const int32_t* offs, int32_t* keys2, int32_t* vals2, int64_t cap,
                           int32_t* flag, int32_t* npairs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl)
        return;
    const int64_t l = perm[i];
    int tl[3][2], nt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        nt[a] = axis_tiles<P>(g, a, base[3 * l + a], tl[a]);
    int64_t pos = offs[i];
    for (int k = 0; k < nt[2]; ++k)
        for (int j = 0; j < nt[1]; ++j)
            for (int q = 0; q < nt[0]; ++q) {
                if (pos < cap) {
                    keys2[pos] = tl[0][q] + g.nt[0] * (tl[1][j] + g.nt[1] * tl[2][k]);
                    vals2[pos] = (int32_t)i;
                } else {
                    flag[1] = 1;
                }
                ++pos;
            }
    if (i == nl - 1)
        npairs[0] = (int32_t)(pos < cap ? pos : cap);
}

// cnt[t'][d]: markers owned by tile t' whose stencil touches tile t' + d;
// tot[t' + d] += that count.  One wavefront per owning tile.  flag[0] counts
// the markers whose dmask entry has bit 31 (stencil leaving the coverage).
__global__ void __launch_bounds__(64)
k_dir_counts(Grid g, int64_t T, const int32_t* __restrict__ tile_offs,
             const int32_t* __restrict__ perm, const uint32_t* __restrict__ dmask,
             int32_t* __restrict__ cnt, int32_t* __restrict__ tot, int32_t* __restrict__ flag)
{
    const int lane = threadIdx.x;
    int nbad = 0;
    for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
        const int s0 = tile_offs[t], s1 = tile_offs[t + 1];
        int mine = 0;                  // lane d < 27: count of direction d
        for (int i0 = s0; i0 < s1; i0 += 64) {
            const int i = i0 + lane;
            const uint32_t m = i < s1 ? dmask[perm[i]] : 0u;
            for (int d = 0; d < NDIR; ++d) {
                const int c = __popcll(__ballot((m >> d) & 1));
                if (lane == d)
                    mine += c;
            }
            nbad += __popcll(__ballot(m >> 31));
        }
        if (lane < NDIR) {
            cnt[t * NDIR + lane] = mine;
            if (mine) {
                int tc[3];
                tile_xyz(g, t, tc);
                atomicAdd(&tot[dir_tile(g, tc, lane, 1)], mine);
            }
        }
    }
    if (lane == 0 && nbad)
        atomicAdd(&flag[0], nbad);
}

// In place: cnt[t'][d] becomes the first position of that run in src_idx
// (the runs of tile t follow src_offs[t] in increasing owner index); every
// entry belongs to exactly one receiving tile.  One wavefront per receiving
// tile (four per workgroup), lane d for direction d; the wavefront of t = T
// clamps the total to the capacity
// and raises flag[1] on overflow.  src_offs[t] is clamped likewise.  A tile
// that no stencil reaches (tot[t] = 0) has only empty runs, which the emit
// pass never reads: their entries keep their (zero) counts.
__global__ void __launch_bounds__(256)
k_dir_offsets(Grid g, int64_t T, int32_t* __restrict__ cnt, int32_t* __restrict__ src_offs,
              const int32_t* __restrict__ tot, int64_t cap, int32_t* __restrict__ flag)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t > T)
        return;
    const int o = src_offs[t];
    if (t == T) {
        if (lane == 0 && o > cap) {
            flag[1] = 1;
            src_offs[T] = (int32_t)cap;
        }
        return;
    }
    if (lane == 0 && o > cap)
        src_offs[t] = (int32_t)cap;
    if (tot[t] == 0)
        return;
    int tc[3];
    tile_xyz(g, t, tc);
    int own = -1, c = 0;
    if (lane < NDIR) {
        const int64_t ow = dir_tile(g, tc, lane, -1);
        if (ow >= 0) {
            own = (int)ow;
            c = cnt[ow * NDIR + lane];
        }
    }
    int pos = o;
    for (int e = 0; e < NDIR; ++e) {
        const int oe = __builtin_amdgcn_readlane(own, e);
        const int ce = __builtin_amdgcn_readlane(c, e);
        pos += (unsigned)oe < (unsigned)own ? ce : 0;
    }
    if (own >= 0)
        cnt[(int64_t)own * NDIR + lane] = pos;
}

// Each owning tile writes its runs: marker i goes to position first + rank in
// every run its stencil touches (rank = earlier markers of the tile in that
// run).  Positions past the capacity are dropped (flag[1] is raised).
__global__ void __launch_bounds__(64)
k_dir_emit(Grid g, int64_t T, const int32_t* __restrict__ tile_offs,
           const int32_t* __restrict__ perm, const uint32_t* __restrict__ dmask,
           const int32_t* __restrict__ first, int32_t* __restrict__ src_idx, int64_t cap)
{
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
        const int s0 = tile_offs[t], s1 = tile_offs[t + 1];
        if (s0 == s1)
            continue;
        int next = lane < NDIR ? first[t * NDIR + lane] : 0;   // lane d: run d's next slot
        for (int i0 = s0; i0 < s1; i0 += 64) {
            const int i = i0 + lane;
            const uint32_t m = i < s1 ? dmask[perm[i]] : 0u;
            for (int d = 0; d < NDIR; ++d) {
                const uint64_t bd = __ballot((m >> d) & 1);
                if (!bd)
                    continue;
                const int start = __builtin_amdgcn_readlane(next, d);
                if ((m >> d) & 1) {
                    const int64_t pos =
                        (int64_t)start +
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(bd >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bd, 0u));
                    if (pos < cap)
                        src_idx[pos] = i;
                }
                if (lane == d)
                    next += __popcll(bd);
            }
        }
    }
}

static int key_bits(int64_t T)
{
    int bits = 0;
    while (((int64_t)1 << bits) < T)
        ++bits;
    return bits;
}

struct BucketWs {
    int32_t *keys, *tk, *tv, *cnt, *total, *npairs, *keys2, *tk2, *tv2;
    int32_t *dcnt, *dtot;   // [T][27] run counts, then run starts; [T] list lengths
    uint32_t* dmask;        // [nl] directions of the tiles each marker's stencil touches
    void *rs, *scan, *dscan;
};

// Source lists by direction need every axis to hold at least 3 tiles.
static bool by_direction(const Grid& g)
{
    return g.nt[0] >= 3 && g.nt[1] >= 3 && g.nt[2] >= 3;
}

static BucketWs carve_bucket_ws(void* ws, size_t bytes, int64_t nl, int64_t cap, int64_t Tdir,
                                size_t* need)
{
    Carver cv(ws, bytes);
    BucketWs w;
    w.dcnt = cv.take<int32_t>(NDIR * Tdir);
    w.dtot = cv.take<int32_t>(Tdir);
    w.dscan = cv.take<char>(scan_workspace(Tdir));
    w.dmask = cv.take<uint32_t>(Tdir > 0 ? nl : 0);
    w.keys = cv.take<int32_t>(nl);
    w.tk = cv.take<int32_t>(nl);
    w.tv = cv.take<int32_t>(nl);
    w.cnt = cv.take<int32_t>(nl);
    w.total = cv.take<int32_t>(1);
    w.npairs = cv.take<int32_t>(1);
    w.keys2 = cv.take<int32_t>(cap);
    w.tk2 = cv.take<int32_t>(cap);
    w.tv2 = cv.take<int32_t>(cap);
    size_t rsb = radix_workspace(cap > nl ? cap : nl);
    w.rs = cv.take<char>(rsb);
    w.scan = cv.take<char>(scan_workspace(nl));
    *need = cv.used;
    return w;
}

}  // namespace ibx

using namespace ibx;

extern "C" size_t ib_bucket_workspace(const ib_level* lv, int64_t nl)
{
    size_t need = 0;
    if (nl < 0 || check_level(lv))
        return 0;
    const Grid g = make_grid(lv);
    carve_bucket_ws(nullptr, 0, nl, 8 * (nl > 0 ? nl : 1), by_direction(g) ? g.ntiles : 0,
                    &need);
    return need;
}

extern "C" int ib_bucket(const ib_level* lv, const ib_markers* m, ib_delta delta,
                         const ib_buckets* b, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_level(lv);
    if (rc)
        return rc;
    if (!m || !b || (delta != IB_DELTA3 && delta != IB_DELTA4) || m->nl < 0 ||
        m->nl > (int64_t)INT32_MAX / 8)
        return IB_EINVAL;
    if (!b->tile_offs || !b->src_offs || !b->flag)
        return IB_EINVAL;
    const int64_t nl = m->nl;
    if (nl > 0 && (!m->x || !m->y || !m->z || !b->cell || !b->tileid || !b->base || !b->perm ||
                   !b->src_idx || b->src_cap < 0))
        return IB_EINVAL;
    Grid g = make_grid(lv);
    const int64_t T = g.ntiles;
    hipStream_t st = (hipStream_t)stream;
    size_t need = 0;
    const int64_t cap = b->src_cap < 8 * nl ? b->src_cap : 8 * nl;
    const bool dir = by_direction(g);
    BucketWs w = carve_bucket_ws(nullptr, 0, nl, cap, dir ? T : 0, &need);
    if (!ws || ws_bytes < need)
        return IB_EWORKSPACE;
    w = carve_bucket_ws(ws, ws_bytes, nl, cap, dir ? T : 0, &need);

    // the flags (and, for lists by direction, their totals) start cleared:
    // here, or with lists by direction in the key kernel
    if (nl == 0 || !dir)
        k_init_flags<<<1, 256, 0, st>>>(b->flag, 0, w.dtot);
    if (nl == 0) {
        lower_bounds(w.keys, 0, nullptr, b->tile_offs, T, st);
        lower_bounds(w.keys, 0, nullptr, b->src_offs, T, st);
        return launch_status();
    }
    const unsigned gb = (unsigned)((nl + 255) / 256);
    const int bits = key_bits(T);
    const int passes = (bits + 7) / 8;
    const int kb = 8 * passes + 4 <= 31 ? 8 * passes : 0;   // 4 count bits above the digits
    const int64_t nz = dir ? T : 0;      // the list totals, when used
    if (delta == IB_DELTA3)
        k_bucket_keys<3><<<gb, 256, 0, st>>>(g, nl, m->x, m->y, m->z, b->cell, b->tileid,
                                             b->base, w.keys, b->perm, b->flag, kb,
                                             dir ? w.dmask : nullptr, nz, w.dtot);
    else
        k_bucket_keys<4><<<gb, 256, 0, st>>>(g, nl, m->x, m->y, m->z, b->cell, b->tileid,
                                             b->base, w.keys, b->perm, b->flag, kb,
                                             dir ? w.dmask : nullptr, nz, w.dtot);
    radix_sort_pairs(w.keys, b->perm, w.tk, w.tv, nl, nullptr, bits, w.rs, st);
    lower_bounds(w.keys, nl, nullptr, b->tile_offs, T, st, kb > 0 ? (1 << kb) - 1 : -1);

    if (dir) {
        const unsigned gw = (unsigned)(T < 16384 ? T : 16384);
        k_dir_counts<<<gw, 64, 0, st>>>(g, T, b->tile_offs, b->perm, w.dmask, w.dcnt, w.dtot,
                                        b->flag);
        scan_exclusive(w.dtot, b->src_offs, T, b->src_offs + T, w.dscan, st);
        k_dir_offsets<<<(unsigned)((T + 4) / 4), 256, 0, st>>>(g, T, w.dcnt, b->src_offs,
                                                              w.dtot, cap, b->flag);
        k_dir_emit<<<gw, 64, 0, st>>>(g, T, b->tile_offs, b->perm, w.dmask, w.dcnt, b->src_idx,
                                      cap);
        return launch_status();
    }

    if (kb > 0) {
        scan_exclusive(w.keys, w.cnt, nl, nullptr, w.scan, st, kb);
    } else {
        if (delta == IB_DELTA3)
            k_src_count<3><<<gb, 256, 0, st>>>(g, nl, b->perm, b->base, w.cnt);
        else
            k_src_count<4><<<gb, 256, 0, st>>>(g, nl, b->perm, b->base, w.cnt);
        scan_exclusive(w.cnt, w.cnt, nl, nullptr, w.scan, st);
    }
    if (delta == IB_DELTA3)
        k_src_emit<3><<<gb, 256, 0, st>>>(g, nl, b->perm, b->base, w.cnt, w.keys2, b->src_idx,
                                          cap, b->flag, w.npairs);
    else
        k_src_emit<4><<<gb, 256, 0, st>>>(g, nl, b->perm, b->base, w.cnt, w.keys2, b->src_idx,
                                          cap, b->flag, w.npairs);
    radix_sort_pairs(w.keys2, b->src_idx, w.tk2, w.tv2, cap, w.npairs, bits, w.rs, st);
    lower_bounds(w.keys2, cap, w.npairs, b->src_offs, T, st);
    return launch_status();
}
