// tiles.h -- the tile-staged interpolation and spreading kernels of the
// batched path (included by batched.hip only).
//
// Interpolation (one work item = up to bw markers of one 8^3 tile): the
// tile plus a ceil(P/2)-cell halo of the field is staged into LDS as one
// 4-vector per cell.  Addresses come from small per-item tables (per-axis
// wrapped coordinates and the ids of the <= 3 boxes or tiles the halo spans
// along each axis), so staging issues independent loads with no division or
// dependent lookups per cell.  One thread per marker then sums its P^3
// stencil from LDS.
//
// Spreading (one work item = one tile with a non-empty source list, one
// wavefront): lane = source marker.  For every stencil offset each lane does
// a plain LDS read-modify-write of its cell.  In one instruction two lanes
// touch the same cell only if their markers share the stencil base cell, so
// lanes are ranked among equal bases (ballot matching on the base key) and
// rank classes are processed one after another.  No atomics; every cell's
// sum is formed in a fixed order (source chunk, rank, offset), so results are
// reproducible bit for bit.
#pragma once

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

// mode 0: field = u0 (box layout): D = (U^d - J u0)/dt, F = D.
// mode 1: field = G (slots): F += D - J G.
// mode 2: field = G (slots): residual only.
// e2 (nullable) receives dV |U^d - J u^(m)|^2 per marker.
template <typename T, int P, int MODE>
__global__ void __launch_bounds__(256)
k_interp_tiles(Grid g, int64_t nl, double dt, const Item* __restrict__ items,
               const int32_t* __restrict__ nitems, const T* __restrict__ u0,
               const T* __restrict__ G, const int32_t* __restrict__ slot, MarkerSoA<T, P> s,
               double* __restrict__ e2)
{
    using V4 = typename Vec4<T>::type;
    constexpr int gh = Halo<P>::g, R = Halo<P>::R, R3 = Halo<P>::R3;
    __shared__ V4 fld[R3];
    __shared__ int32_t ax_off[3][R];   // per-axis part of the element offset
    __shared__ int32_t ax_sel[3][R];   // which box / tile along the axis (-1: outside)
    __shared__ int64_t nb_base[27];    // element offset of each (box or tile) or -1
    const int n_items = *nitems;
    const double h3 = g.h * g.h * g.h;
    const int tid = threadIdx.x;
    const int64_t comp = MODE == 0 ? g.cstride : (int64_t)TILE_CELLS;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = items[it];
        int lo[3];
        tile_coords(g, item.tile, lo);
        // per-axis tables
        const int unit = MODE == 0 ? g.box : TILE;
        if (tid < 3 * R) {
            const int a = tid / R, j = tid - a * R;
            // selector = number of unit changes along the axis up to cell j
            int sel = 0, prev = 0, c = 0, ok = 1;
            for (int q = 0; q <= j; ++q) {
                c = lo[a] - gh + q;
                ok = 1;
                if (c < 0) {
                    if (g.periodic[a]) c += g.n[a]; else ok = 0;
                } else if (c >= g.n[a]) {
                    if (g.periodic[a]) c -= g.n[a]; else ok = 0;
                }
                const int u = ok ? c / unit : -1;
                if (q > 0 && u != prev)
                    ++sel;
                prev = u;
            }
            const int l = ok ? c - (c / unit) * unit : 0;
            int off;
            if (MODE == 0) {
                const int e = l + g.ngrow;
                off = a == 0 ? e : (a == 1 ? e * g.ext : e * g.ext * g.ext);
            } else {
                off = a == 0 ? l : (a == 1 ? l * TILE : l * TILE * TILE);
            }
            ax_off[a][j] = off;
            ax_sel[a][j] = ok ? sel : -1;
        }
        __syncthreads();
        if (tid < 27) {
            const int sv[3] = {tid % 3, (tid / 3) % 3, tid / 9};
            int u[3];
            bool have = true;
            for (int a = 0; a < 3; ++a) {
                int j0 = -1;
                for (int j = 0; j < R; ++j)
                    if (ax_sel[a][j] == sv[a]) {
                        j0 = j;
                        break;
                    }
                if (j0 < 0) {
                    have = false;
                    u[a] = 0;
                } else {
                    int c = lo[a] - gh + j0;
                    if (c < 0) c += g.n[a];
                    else if (c >= g.n[a]) c -= g.n[a];
                    u[a] = c / unit;
                }
            }
            int64_t base = -1;
            if (have) {
                const int ux = u[0], uy = u[1], uz = u[2];
                if (MODE == 0) {
                    const int id = g.lut[ux + g.nb[0] * (uy + g.nb[1] * uz)];
                    base = id >= 0 ? (int64_t)id * g.bstride : -1;
                } else {
                    const int sl = slot[ux + g.nt[0] * (uy + g.nt[1] * uz)];
                    base = sl >= 0 ? (int64_t)sl * 3 * TILE_CELLS : -1;
                }
            }
            nb_base[tid] = base;
        }
        __syncthreads();
        // stage the tile and its halo
        for (int q = tid; q < R3; q += blockDim.x) {
            const int jx = q % R, jy = (q / R) % R, jz = q / (R * R);
            const int sx = ax_sel[0][jx], sy = ax_sel[1][jy], sz = ax_sel[2][jz];
            V4 v;
            v.x = T(0);
            v.y = T(0);
            v.z = T(0);
            v.w = T(0);
            if ((sx | sy | sz) >= 0) {
                const int64_t b = nb_base[sx + 3 * (sy + 3 * sz)];
                if (b >= 0) {
                    const int64_t off = b + ax_off[0][jx] + ax_off[1][jy] + ax_off[2][jz];
                    const T* src = MODE == 0 ? u0 : G;
                    v.x = src[off];
                    v.y = src[off + comp];
                    v.z = src[off + 2 * comp];
                }
            }
            fld[q] = v;
        }
        __syncthreads();
        if (tid < item.count) {
            const int64_t i = item.start + tid;
            int lb[3];
            bool ok = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lb[a] = s.rb[a * nl + i] - lo[a] + gh;
                ok &= (lb[a] >= 0 && lb[a] <= R - P);
            }
            T w[3][P];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int o = 0; o < P; ++o)
                    w[a][o] = s.rw[(a * P + o) * nl + i];
            T acc0 = 0, acc1 = 0, acc2 = 0;
            if (ok) {
#pragma unroll
                for (int k = 0; k < P; ++k)
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const T wyz = w[1][j] * w[2][k];
                        const int row = ((lb[2] + k) * R + (lb[1] + j)) * R + lb[0];
#pragma unroll
                        for (int q = 0; q < P; ++q) {
                            const T wt = w[0][q] * wyz;
                            const V4 v = fld[row + q];
                            acc0 += v.x * wt;
                            acc1 += v.y * wt;
                            acc2 += v.z * wt;
                        }
                    }
            }
            const T acc[3] = {acc0, acc1, acc2};
            double err = 0.0;
            const T idt = (T)(1.0 / dt);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (MODE == 0) {
                    const T e = s.ud[c * nl + i] - acc[c];
                    const T dd = e * idt;
                    s.d[c * nl + i] = dd;
                    s.fs[c * nl + i] = dd;
                    err += (double)e * (double)e;
                } else {
                    const T r = s.d[c * nl + i] - acc[c];   // = (U^d - J u^(m))/dt
                    if (MODE == 1)
                        s.fs[c * nl + i] = s.fs[c * nl + i] + r;
                    const double e = (double)r * dt;
                    err += e * e;
                }
            }
            if (e2)
                e2[i] = (double)s.rs[i] * h3 * err;
        }
        __syncthreads();
    }
}

// One wavefront per workgroup.  FINAL = 0: store the tile to its G slot.
// FINAL = 1: store f (if any) and ustar = u0 + dt G on the tile; also the G
// slot when keep_g is set (final residual).
template <typename T, int P, int FINAL>
__global__ void __launch_bounds__(64)
k_spread_tiles(Grid g, int64_t nl, double dt, const int32_t* __restrict__ active,
               const int32_t* __restrict__ nactive, const int32_t* __restrict__ src_offs,
               const int32_t* __restrict__ src_idx, MarkerSoA<T, P> s, T* __restrict__ G,
               const T* __restrict__ u0, T* __restrict__ ustar, T* __restrict__ f, int keep_g)
{
    using V4 = typename Vec4<T>::type;
    __shared__ V4 acc[TILE_CELLS];
    const int lane = threadIdx.x;
    const uint64_t lt = lane ? ((~0ull) >> (64 - lane)) : 0ull;
    const int n_act = *nactive;
    for (int a = blockIdx.x; a < n_act; a += gridDim.x) {
        const int t = active[a];
        int lo[3];
        tile_coords(g, t, lo);
        for (int q = lane; q < TILE_CELLS; q += 64) {
            V4 z;
            z.x = T(0);
            z.y = T(0);
            z.z = T(0);
            z.w = T(0);
            acc[q] = z;
        }
        __syncthreads();
        const int s0 = src_offs[t], s1 = src_offs[t + 1];
        for (int sb = s0; sb < s1; sb += 64) {
            const int sidx = sb + lane;
            const bool valid = sidx < s1;
            const int64_t i = valid ? src_idx[sidx] : 0;
            // tile-frame coordinates of the stencil cells and their in-tile masks
            int cx[P], cy[P], cz[P];
            int mx = 0, my = 0, mz = 0, key = 0;
            T w[3][P];
            T F0 = 0, F1 = 0, F2 = 0;
            if (valid) {
                int d[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax)
                    d[ax] = wrapi(s.rb[ax * nl + i] - lo[ax], g.n[ax]);
#pragma unroll
                for (int o = 0; o < P; ++o) {
                    int x = d[0] + o, y = d[1] + o, zc = d[2] + o;
                    if (x >= g.n[0]) x -= g.n[0];
                    if (y >= g.n[1]) y -= g.n[1];
                    if (zc >= g.n[2]) zc -= g.n[2];
                    cx[o] = x;
                    cy[o] = y * TILE;
                    cz[o] = zc * TILE * TILE;
                    mx |= (x < TILE) << o;
                    my |= (y < TILE) << o;
                    mz |= (zc < TILE) << o;
                }
                // base key: tile-frame base in [-3, 7] per axis, shifted to [0, 10]
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const int b = d[ax] > g.n[ax] - P ? d[ax] - g.n[ax] : d[ax];
                    key |= (b + 3) << (4 * ax);
                }
#pragma unroll
                for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                    for (int o = 0; o < P; ++o)
                        w[ax][o] = s.rw[(ax * P + o) * nl + i];
                const T sc = s.rs[i];
                F0 = s.fs[0 * nl + i] * sc;
                F1 = s.fs[1 * nl + i] * sc;
                F2 = s.fs[2 * nl + i] * sc;
            } else {
#pragma unroll
                for (int o = 0; o < P; ++o) {
                    cx[o] = cy[o] = cz[o] = 0;
                    w[0][o] = w[1][o] = w[2][o] = T(0);
                }
            }
            // rank among lanes with the same base key
            uint64_t mask = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 12; ++bit) {
                const bool on = (key >> bit) & 1;
                const uint64_t m = __ballot(valid && on);
                mask &= on ? m : ~m;
            }
            const int rank = __popcll(mask & lt);
            int rmax = 0;
            while (__ballot(valid && rank > rmax))
                ++rmax;
#pragma unroll
            for (int k = 0; k < P; ++k)
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const T wyz = w[1][j] * w[2][k];
                    const bool inyz = valid && ((my >> j) & 1) && ((mz >> k) & 1);
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        const bool in = inyz && ((mx >> q) & 1);
                        const T wt = w[0][q] * wyz;
                        const int cell = cx[q] + cy[j] + cz[k];
                        // rank classes in turn: no two active lanes share a cell
                        for (int r = 0; r <= rmax; ++r) {
                            if (in && rank == r) {
                                V4 v = acc[cell];
                                v.x += F0 * wt;
                                v.y += F1 * wt;
                                v.z += F2 * wt;
                                acc[cell] = v;
                            }
                        }
                    }
                }
        }
        __syncthreads();
        if (!FINAL || keep_g) {
            T* gs = G + (int64_t)a * 3 * TILE_CELLS;
            for (int q = lane; q < TILE_CELLS; q += 64) {
                const V4 v = acc[q];
                gs[q] = v.x;
                gs[q + TILE_CELLS] = v.y;
                gs[q + 2 * TILE_CELLS] = v.z;
            }
        }
        if (FINAL) {
            const T tdt = (T)dt;
            for (int q = lane; q < TILE_CELLS; q += 64) {
                const int64_t off = cell_offset(g, lo[0] + (q & 7), lo[1] + ((q >> 3) & 7),
                                                lo[2] + (q >> 6));
                if (off < 0)
                    continue;
                const V4 v = acc[q];
                const T vc[3] = {v.x, v.y, v.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t o = off + c * g.cstride;
                    if (f)
                        f[o] = vc[c];
                    ustar[o] = u0[o] + tdt * vc[c];
                }
            }
        }
        __syncthreads();
    }
}
