// tiles.h -- the tile-staged interpolation and spreading kernels of the
// batched path (included by batched.hip only).  Every axis of the grid has
// at least 16 cells here, so a stencil never wraps onto its own tile.
//
// Interpolation (one work item = up to BW markers of one 8^3 tile, BW
// threads): the tile plus a ceil(P/2)-cell halo of the field is staged into
// three LDS planes.  For every item the element offsets of the 27 tiles
// around it are precomputed once per loop (item_base), so a halo cell's
// address is base[(j-g+8)>>3 per axis] + its position in that tile.  Items
// with few markers spread each marker over 2 or 4 lanes (one z plane of the
// stencil each), so all waves of the workgroup share the compute phase.
//
// Spreading (one work item = one tile with a non-empty source list, one
// wavefront): lane = one (y, z) row of the tile, holding its 8 cells x 3
// components in registers.  Sources are staged 64 at a time in LDS; ballots
// give each lane the set of staged sources whose stencil covers its row.
// Rows near a particle surface are covered by several times more sources than
// the mean, so the visits are balanced in two phases: each lane first takes up
// to K sources of its own row, then the rest of the heavier rows is dealt out
// in pieces of K to all lanes and added back by the row's owner in order.  No
// atomics: each cell's sum is formed in a fixed order, so the result is
// reproducible bit for bit.  Each lane then stores its row (8 consecutive
// cells per component in the tile's slot) straight from registers.
#pragma once

// XCD-aware static work split.  Workgroups are dispatched to the 8 XCDs of
// the device round-robin by id, and each XCD has its own L2.  The work list
// (ordered by tile, so consecutive items are spatial neighbours) is cut into
// 8 contiguous slabs and the workgroups of XCD x stride over slab x, so the
// halo cells shared by neighbouring items are fetched into one L2, not eight.
// The grid is a multiple of 8 workgroups.  Which workgroup computes an item
// never changes the item's result.
constexpr int NXCD = 8;

struct Slab {
    int begin, end, stride;
};

__device__ inline Slab xcd_slab(int n)
{
    const int per = (n + NXCD - 1) / NXCD;
    const int x = blockIdx.x % NXCD;
    Slab r;
    r.begin = x * per + (int)(blockIdx.x / NXCD);
    r.end = min(n, (x + 1) * per);
    r.stride = gridDim.x / NXCD;
    return r;
}

// Element offsets of the 9 NBX tiles around an interpolation item (NBX
// along x: the work tile's own TXW / 8 tiles and one on each side; 3 along y
// and z), for an item of work tile t and neighbour k < 9 NBX: *bu in the
// velocity field (box layout), *bg in the per-tile force buffer.  -1 where
// the tile lies outside a bounded axis, in an uncovered box, or has no force
// slot (a tile has one when its source list is not empty: slot act_offs[tile]).
template <int NBX>
__device__ inline void item_base(const Grid& g, int t, int k, const int32_t* __restrict__ src_offs,
                                 const int32_t* __restrict__ act_offs, int64_t* bu, int64_t* bg)
{
    int lo[3];
    lo[0] = (t % g.nt[0]) * TILE;
    lo[1] = ((t / g.nt[0]) % g.nt[1]) * TILE;
    lo[2] = (t / (g.nt[0] * g.nt[1])) * TILE;
    const int sel[3] = {k % NBX, (k / NBX) % 3, k / (3 * NBX)};
    int c[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        int v = lo[a] + (sel[a] - 1) * TILE;
        if (v < 0) {
            if (g.periodic[a]) v += g.n[a]; else ok = false;
        } else if (v >= g.n[a]) {
            if (g.periodic[a]) v -= g.n[a]; else ok = false;
        }
        c[a] = v;
    }
    *bu = *bg = -1;
    if (ok) {
        *bu = cell_offset(g, c[0], c[1], c[2]);
        const int tn = (c[0] >> 3) + g.nt[0] * ((c[1] >> 3) + g.nt[1] * (c[2] >> 3));
        if (src_offs[tn + 1] > src_offs[tn])
            *bg = (int64_t)act_offs[tn] * 3 * TILE_CELLS;
    }
}

// mode 0: field = u0 (box layout): D = (U^d - J u0)/dt, F = D.
// mode 1: field = G (slots): F += D - J G.
// mode 2: field = G (slots): residual only.
// mode 3: field = u0 (any field in the box layout), for the adjoint:
//         Fout[l] = J field (if Fout) and gX[l] += sc sum over the stencil of
//         (field . vin_l) grad_X w_l, sc = dV/h^3 (use_dv) or 1, in marker
//         order (the weights' derivatives from the same shared root).
// e2 (nullable) receives dV |U^d - J u^(m)|^2 per marker.
// (FP32 with the row masks, 256-marker items of one tile: registers capped at
// the unmasked kernel's seven waves per SIMD.)
template <typename T, int P, int MODE, int BW, bool MASK = false, int TXW = TILE>
__global__ void __launch_bounds__(BW)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && BW == 256 && TXW == TILE
                                        ? (MASK ? 7 : MODE == 0 ? 5 : 1) : 1, 8)))
k_interp_tiles(Grid g, int64_t nl, double dt, const Item* __restrict__ items,
               const int32_t* __restrict__ nitems, const T* __restrict__ u0,
               const T* __restrict__ G, const int64_t* __restrict__ nbase, MarkerData<T> s,
               double* __restrict__ e2, T* __restrict__ Fout, const int32_t* __restrict__ perm,
               const T* __restrict__ vin, double* __restrict__ gX, int use_dv,
               const uint64_t* __restrict__ rmask)
{
    constexpr bool BOX = MODE == 0 || MODE == 3;   // field in the box layout
    constexpr int gh = Halo<P>::g, R = Halo<P>::R;
    // The work tile is TXW x 8 x 8 cells: one tile, or two x neighbours
    // (TXW = 16).  LDS holds its halo as rows [c][jz][jy] of pitch RP with
    // halo x index jx at position jx + XO, so the tile's own cells sit at
    // 2 .. TXW + 1 and every row segment lands on an aligned pair boundary.
    // NBX tiles along x (the TXW / 8 own ones and one on each side), 3 along
    // y and z, hold the halo.
    constexpr int RX = TXW + 2 * gh, RP = TXW == TILE ? 12 : 20, XO = 2 - gh;
    constexpr int PL = R * R * RP, NROW = 3 * R * R;
    constexpr int NBX = TXW / TILE + 2, NNB = 9 * NBX;
    static_assert(TXW == TILE || TXW == 2 * TILE, "work tile of one or two tiles along x");
    static_assert(TXW + 4 <= RP, "a row holds the paired window of TXW + 4 cells");
    using T2 = typename Vec2<T>::type;
    __shared__ __align__(16) T fld[3 * PL];
    __shared__ int64_t nb[NNB];
    __shared__ uint64_t nbm[NNB];       // tile slots: rows of each neighbour's slot not all zero
    const int n_items = *nitems;
    const double h3 = g.h * g.h * g.h;
    const int tid = threadIdx.x;
    const int64_t comp = BOX ? g.cstride : (int64_t)TILE_CELLS;
    const int sy = BOX ? g.ext : TILE;
    const int sz = BOX ? g.ext * g.ext : TILE * TILE;
    const T* src = BOX ? u0 : G;
    // box layout: pair loads need an even ghost width and a field aligned to
    // two elements (box extents and component strides are then even)
    const bool pairs = BOX && (g.ngrow & 1) == 0 && !((uintptr_t)src & (2 * sizeof(T) - 1));
    const Slab sl = xcd_slab(n_items);
    // The neighbour offsets of each item are loaded one item ahead (two with
    // the row masks, whose loads follow them one item ahead), so the staging
    // and compute of an item hide those loads.
    auto row_mask = [&](int64_t off) -> uint64_t {
        return off >= 0 ? rmask[off / (3 * TILE_CELLS)] : 0ull;
    };
    int64_t pnb = sl.begin < sl.end && tid < NNB ? nbase[(int64_t)sl.begin * NNB + tid] : 0;
    uint64_t pm = 0ull;
    int64_t qnb = 0;
    if constexpr (MASK) {
        if (tid < NNB && sl.begin < sl.end)
            pm = row_mask(pnb);
        if (tid < NNB && sl.begin + sl.stride < sl.end)
            qnb = nbase[(int64_t)(sl.begin + sl.stride) * NNB + tid];
    }
    for (int it = sl.begin; it < sl.end; it += sl.stride) {
        if (tid < NNB) {
            nb[tid] = pnb;
            if constexpr (MASK)
                nbm[tid] = pm;
        }
        __syncthreads();
        if constexpr (MASK) {
            if (tid < NNB) {
                pnb = qnb;
                pm = it + sl.stride < sl.end ? row_mask(qnb) : 0ull;
                if (it + 2 * sl.stride < sl.end)
                    qnb = nbase[(int64_t)(it + 2 * sl.stride) * NNB + tid];
            }
        } else if (tid < NNB && it + sl.stride < sl.end) {
            pnb = nbase[(int64_t)(it + sl.stride) * NNB + tid];
        }
        const Item item = items[it];
        int lo[3];
        tile_coords(g, item.tile, lo);
        // Marker records are fetched just before the halo so both streams of
        // loads are in flight together.  Small items spread each marker over
        // `split` consecutive lanes, one z plane of the stencil per lane (then
        // a shuffle sum), so every wave of the workgroup takes part in the
        // compute phase.
        const int cnt = item.count;
        const int lg = 4 * cnt <= BW ? 2 : 2 * cnt <= BW ? 1 : 0;
        const int split = 1 << lg;
        const int sub = tid & (split - 1);
        const bool mine = (tid >> lg) < cnt;
        const int64_t i = item.start + (mine ? (tid >> lg) : 0);
        int lb[3];
        T w[3][P], dw[3][P];
        T dd[3] = {T(0), T(0), T(0)};
        T vv[3] = {T(0), T(0), T(0)};
        T rs = T(0);
        typename Vec4<T>::type fv;
        fv.x = fv.y = fv.z = fv.w = T(0);
        if (mine) {
            const typename Vec4<T>::type gq = s.geo[i];
            int rb[3];
            unpack_rb(s.rb[i], rb);
            if (MODE == 3) {
                axis_weights_rd<T, P>(gq.x, w[0], dw[0]);
                axis_weights_rd<T, P>(gq.y, w[1], dw[1]);
                axis_weights_rd<T, P>(gq.z, w[2], dw[2]);
                const int64_t l = perm[i];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    vv[c] = vin[3 * l + c];
            } else {
                axis_weights_r<T, P>(gq.x, w[0]);
                axis_weights_r<T, P>(gq.y, w[1]);
                axis_weights_r<T, P>(gq.z, w[2]);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
                lb[a] = rb[a] - lo[a] + gh;
            rs = gq.w;
            if (sub == 0 && MODE != 3) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    dd[c] = MODE == 0 ? s.ud[c * nl + i] : s.d[c * nl + i];
                if (MODE == 1)
                    fv = s.f4[i];
            }
        }
        if (BOX && pairs) {
            // box layout with an even ghost width: every tile starts on an
            // even element, so the window lo - 2 .. lo + TXW + 1 of each row
            // (the halo of either kernel width) moves in aligned x pairs, none
            // across a tile; consecutive lanes take consecutive pairs
            constexpr int NPR = TXW / 2 + 2, R2 = NPR * R * R, NPT = (R2 + BW - 1) / BW;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int q = tid + k * BW;
                if (q < R2) {
                    const int px = q % NPR, jy = (q / NPR) % R, jz = q / (NPR * R);
                    const int xo = 2 * px - 2;   // x of the pair's first cell from lo
                    const int sel = ((xo + TILE) >> 3) + NBX * (((jy - gh + TILE) >> 3) +
                                                                3 * ((jz - gh + TILE) >> 3));
                    const int64_t b = nb[sel];
                    T2 v0, v1, v2;
                    v0.x = v0.y = v1.x = v1.y = v2.x = v2.y = T(0);
                    if (b >= 0) {
                        const T* p = src + b + (xo & 7) + (int64_t)sy * ((jy - gh) & 7) +
                                     (int64_t)sz * ((jz - gh) & 7);
                        v0 = *reinterpret_cast<const T2*>(p);
                        v1 = *reinterpret_cast<const T2*>(p + comp);
                        v2 = *reinterpret_cast<const T2*>(p + 2 * comp);
                    }
                    const int at = (jz * R + jy) * RP + 2 * px;
                    *reinterpret_cast<T2*>(fld + at) = v0;
                    *reinterpret_cast<T2*>(fld + PL + at) = v1;
                    *reinterpret_cast<T2*>(fld + 2 * PL + at) = v2;
                }
            }
        } else if (BOX) {
            // box layout, odd ghost width: consecutive lanes take consecutive
            // cells of the halo
            constexpr int R3 = RX * R * R, NPT = (R3 + BW - 1) / BW;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int q = tid + k * BW;
                if (q < R3) {
                    const int jx = q % RX, jy = (q / RX) % R, jz = q / (RX * R);
                    const int sel = ((jx - gh + TILE) >> 3) + NBX * (((jy - gh + TILE) >> 3) +
                                                                    3 * ((jz - gh + TILE) >> 3));
                    const int64_t b = nb[sel];
                    T v0 = T(0), v1 = T(0), v2 = T(0);
                    if (b >= 0) {
                        const int64_t off = b + ((jx - gh) & 7) + (int64_t)sy * ((jy - gh) & 7) +
                                            (int64_t)sz * ((jz - gh) & 7);
                        v0 = src[off];
                        v1 = src[off + comp];
                        v2 = src[off + 2 * comp];
                    }
                    const int at = (jz * R + jy) * RP + XO + jx;
                    fld[at] = v0;
                    fld[PL + at] = v1;
                    fld[2 * PL + at] = v2;
                }
            }
        }
        // tile slots (rows start on multiples of 8 elements, so they move in
        // pairs): stage the halo row by row -- left segment (gh cells of the
        // -x neighbour), the 8 cells of each own tile, right segment
        for (int task = tid; !BOX && task < NROW; task += BW) {
            const int c = task / (R * R), rr = task - c * (R * R);
            const int jy = rr % R, jz = rr / R;
            const int ys = (jy - gh + TILE) >> 3, zs = (jz - gh + TILE) >> 3;
            const int64_t roff = (int64_t)sy * ((jy - gh) & 7) + (int64_t)sz * ((jz - gh) & 7) +
                                 c * comp;
            const int q0 = NBX * (ys + 3 * zs);
            int64_t bn[NBX];
#pragma unroll
            for (int x = 0; x < NBX; ++x)
                bn[x] = nb[q0 + x];
            if constexpr (MASK) {
                // a neighbour row whose mask bit is clear is all zeros in its slot
                const int rbit = ((jy - gh) & 7) + TILE * ((jz - gh) & 7);
#pragma unroll
                for (int x = 0; x < NBX; ++x)
                    bn[x] = (nbm[q0 + x] >> rbit) & 1 ? bn[x] : -1;
            }
            T* row = fld + ((c * R + jz) * R + jy) * RP;
            // every load of the row is issued before its first store
            const int64_t bl = bn[0], br = bn[NBX - 1];
            T2 v[TXW / 2];
#pragma unroll
            for (int mt = 0; mt < TXW / TILE; ++mt) {
                const int64_t bc = bn[1 + mt];
                if (bc >= 0) {
                    const T2* q = reinterpret_cast<const T2*>(src + bc + roff);
#pragma unroll
                    for (int k = 0; k < TILE / 2; ++k)
                        v[mt * (TILE / 2) + k] = q[k];
                } else {
#pragma unroll
                    for (int k = 0; k < TILE / 2; ++k)
                        v[mt * (TILE / 2) + k].x = v[mt * (TILE / 2) + k].y = T(0);
                }
            }
            T2 vl, vr;
            vl.x = vl.y = vr.x = vr.y = T(0);
            if (gh == 2) {
                if (bl >= 0)
                    vl = *reinterpret_cast<const T2*>(src + bl + roff + (TILE - 2));
                if (br >= 0)
                    vr = *reinterpret_cast<const T2*>(src + br + roff);
            } else {
                vl.x = bl >= 0 ? src[bl + roff + TILE - 1] : T(0);
                vr.x = br >= 0 ? src[br + roff] : T(0);
            }
#pragma unroll
            for (int k = 0; k < TXW / 2; ++k)
                *reinterpret_cast<T2*>(row + 2 + 2 * k) = v[k];
            if (gh == 2) {
                *reinterpret_cast<T2*>(row) = vl;
                *reinterpret_cast<T2*>(row + 2 + TXW) = vr;
            } else {
                row[XO] = vl.x;
                row[2 + TXW] = vr.x;
            }
        }
        __syncthreads();
        T acc0 = 0, acc1 = 0, acc2 = 0;
        T gr0 = 0, gr1 = 0, gr2 = 0;      // mode 3: position gradient
        if (mine) {
            const bool ok = lb[0] >= 0 && lb[0] <= RX - P && lb[1] >= 0 && lb[1] <= R - P &&
                            lb[2] >= 0 && lb[2] <= R - P;
            // planes sub, sub + split, ...: the trip count is uniform per item
            const int trips = (P + split - 1) >> lg;
            for (int n = 0; n < trips; ++n) {
                const int k = sub + (n << lg);
                if (!ok || k >= P)
                    continue;
                T wz = w[2][0], dwz = MODE == 3 ? dw[2][0] : T(0);
#pragma unroll
                for (int o = 1; o < P; ++o) {
                    wz = k == o ? w[2][o] : wz;
                    if (MODE == 3)
                        dwz = k == o ? dw[2][o] : dwz;
                }
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const T wyz = w[1][j] * wz;
                    const int row = ((lb[2] + k) * R + (lb[1] + j)) * RP + XO + lb[0];
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        const T wt = w[0][q] * wyz;
                        const T f0 = fld[row + q], f1 = fld[PL + row + q],
                                f2 = fld[2 * PL + row + q];
                        acc0 += f0 * wt;
                        acc1 += f1 * wt;
                        acc2 += f2 * wt;
                        if (MODE == 3) {
                            const T dot = f0 * vv[0] + f1 * vv[1] + f2 * vv[2];
                            gr0 += dot * dw[0][q] * wyz;
                            gr1 += dot * w[0][q] * dw[1][j] * wz;
                            gr2 += dot * w[0][q] * w[1][j] * dwz;
                        }
                    }
                }
            }
        }
        if (lg >= 1) {
            acc0 += __shfl_xor(acc0, 1);
            acc1 += __shfl_xor(acc1, 1);
            acc2 += __shfl_xor(acc2, 1);
            if (MODE == 3) {
                gr0 += __shfl_xor(gr0, 1);
                gr1 += __shfl_xor(gr1, 1);
                gr2 += __shfl_xor(gr2, 1);
            }
        }
        if (lg >= 2) {
            acc0 += __shfl_xor(acc0, 2);
            acc1 += __shfl_xor(acc1, 2);
            acc2 += __shfl_xor(acc2, 2);
            if (MODE == 3) {
                gr0 += __shfl_xor(gr0, 2);
                gr1 += __shfl_xor(gr1, 2);
                gr2 += __shfl_xor(gr2, 2);
            }
        }
        if (MODE == 3 && mine && sub == 0) {
            const int64_t l = perm[i];
            if (Fout) {
                Fout[3 * l + 0] = acc0;
                Fout[3 * l + 1] = acc1;
                Fout[3 * l + 2] = acc2;
            }
            // d/dX = (d/ds) / h
            const double sc = (use_dv ? (double)rs : 1.0) / g.h;
            gX[3 * l + 0] += sc * (double)gr0;
            gX[3 * l + 1] += sc * (double)gr1;
            gX[3 * l + 2] += sc * (double)gr2;
        }
        if (MODE != 3 && mine && sub == 0) {
            const T acc[3] = {acc0, acc1, acc2};
            double err = 0.0;
            const T idt = (T)(1.0 / dt);
            T nf[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (MODE == 0) {
                    const T e = dd[c] - acc[c];             // U^d - J u0
                    const T dv = e * idt;
                    s.d[c * nl + i] = dv;
                    nf[c] = dv;
                    err += (double)e * (double)e;
                } else {
                    const T r = dd[c] - acc[c];             // (U^d - J u^(m))/dt
                    nf[c] = r;
                    const double e = (double)r * dt;
                    err += e * e;
                }
            }
            if (MODE == 0) {
                fv.x = nf[0];
                fv.y = nf[1];
                fv.z = nf[2];
                fv.w = T(0);
                s.f4[i] = fv;
            } else if (MODE == 1) {
                fv.x += nf[0];
                fv.y += nf[1];
                fv.z += nf[2];
                s.f4[i] = fv;
            }
            if (MODE != 2 && Fout) {            // the last F, straight to marker order
                const int64_t l = perm[i];
                Fout[3 * l + 0] = fv.x;
                Fout[3 * l + 1] = fv.y;
                Fout[3 * l + 2] = fv.z;
            }
            if (e2)
                e2[i] = (double)rs * h3 * err;
        }
        __syncthreads();
    }
}

// floor(a / b) for 0 <= a < 128, 1 <= b <= 128: the quotient's distance to
// the next integer is at least 1/b unless it is exact, far above the error
// of the single-precision product, so a small bias makes the floor exact.
__device__ inline int small_div(int a, int b)
{
    return (int)((float)a * __builtin_amdgcn_rcpf((float)b) + 1.0e-3f);
}

// Wavefront sums, maxima and prefix sums of small non-negative values
// (below 128) from seven ballots: bit b of the result gathers 2^b times the
// number of lanes with bit b set.  No cross-lane data movement.
__device__ inline int wave_sum(int v)
{
    int s = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b)
        s += __popcll(__ballot((v >> b) & 1)) << b;
    return s;
}

__device__ inline int wave_max(int v)
{
    int m = 0;
#pragma unroll
    for (int b = 6; b >= 0; --b) {
        const int c = m | (1 << b);
        if (__ballot(v >= c))
            m = c;
    }
    return m;
}

__device__ inline int wave_exclusive_sum(int v)
{
    int s = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        const uint64_t bb = __ballot((v >> b) & 1);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
        s += below << b;
    }
    return s;
}

// m with its s lowest set bits cleared (s below the popcount of m): a binary
// search for the position of the s-th set bit by halves, in constant time.
__device__ inline uint64_t drop_low_bits(uint64_t m, int s)
{
    int p = 0;
    uint64_t w = m;
    int c = __popc((uint32_t)w);
    if (s >= c) { s -= c; w >>= 32; p = 32; }
    uint32_t v = (uint32_t)w;
    c = __popc(v & 0xffffu); if (s >= c) { s -= c; v >>= 16; p += 16; }
    c = __popc(v & 0xffu);   if (s >= c) { s -= c; v >>= 8;  p += 8; }
    c = __popc(v & 0xfu);    if (s >= c) { s -= c; v >>= 4;  p += 4; }
    c = __popc(v & 0x3u);    if (s >= c) { s -= c; v >>= 2;  p += 2; }
    if (s >= (int)(v & 1u)) p += 1;
    return m & (~0ull << p);
}

// One wavefront per workgroup; the tile is stored to its G slot.  The
// workgroups of XCD x (ids = x mod 8) take the entries of slab x of `sent`
// (the x-th of 8 equal cuts, each by decreasing cost) dealt in a snake: with
// W workgroups on the XCD, round r gives its w-th workgroup entry r W + w
// (r even) or r W + W - 1 - w (r odd) of the slab.
//
// Sources are staged 64 at a time as structure-of-arrays in LDS: the weight
// of every tile x cell (zero outside the stencil), the P weights along y and
// along z with the stencil's first row, and F dV/h^3 (F alone when use_dv is
// 0: the transpose of interpolation in the adjoint).  Sixteen ballots give,
// per tile row y and per tile row z, the 64-bit set of staged sources whose
// stencil covers it; a lane's own set is the AND of its two, and the lane
// visits exactly those sources in list order.  Each lane holds one (y, z) row
// of the tile and stores it straight to the slot (rows are contiguous there).
// LDS stays near 5.9 KB so that 24 or more workgroups fit on a CU.
// (FP32: registers capped so that 6 waves fit per SIMD, the residency that the
// latency-bound visit chain wants; at that cap the 4-point kernel spills two
// registers, which costs less than the prefetch of the source indices saves.)
template <typename T, int P, bool MASK = false>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1, 8)))
k_spread_tiles(const int4* __restrict__ sent, const int32_t* __restrict__ nactive,
               const int32_t* __restrict__ src_idx, Grid g, MarkerData<T> s,
               T* __restrict__ G, uint64_t* __restrict__ rmask, uint64_t* __restrict__ tmask,
               int use_dv)
{
    constexpr int NW = TILE + 2 * P + 3;                   // staged values per source
    constexpr int NBUF = NW * 64;
    constexpr int MAXP = NBUF / (3 * TILE) < 64 ? NBUF / (3 * TILE) : 64;   // phase-B pieces
    __shared__ T buf[NBUF];
    __shared__ int2 sb[64];             // k - 64 by, k - 64 bz: tile row r (covered by the
                                        // stencil) reads sy[64 r + .x], sz[64 r + .y]
    T* const sx = buf;                  // [TILE][64] x weight of tile cell x
    T* const sy = buf + TILE * 64;      // [P][64]    y weights
    T* const sz = sy + P * 64;          // [P][64]    z weights
    T* const sf = sz + P * 64;          // [3][64]    F dV / h^3
    __shared__ uint64_t rest[64];       // sources of each row left after phase A
    __shared__ int32_t piece[MAXP];     // phase-B slot -> row | piece << 8
    // add source k's contribution to the 8 cells of row (y, z)
    auto visit = [&](T (&a)[TILE][3], int y, int z, int k) {
        const int2 bb = sb[k];
        const T wyz = sy[y * 64 + bb.x] * sz[z * 64 + bb.y];
        const T c0 = sf[k] * wyz, c1 = sf[64 + k] * wyz, c2 = sf[128 + k] * wyz;
#pragma unroll
        for (int x = 0; x < TILE; ++x) {
            const T wv = sx[x * 64 + k];
            a[x][0] += c0 * wv;
            a[x][1] += c1 * wv;
            a[x][2] += c2 * wv;
        }
    };
    const int lane = threadIdx.x;
    const int ly = lane & 7, lz = lane >> 3;
    const int n_act = *nactive;
    const int per = (n_act + NXCD - 1) / NXCD;
    const int x = blockIdx.x % NXCD, nwg = gridDim.x / NXCD, wg = blockIdx.x / NXCD;
    const int s_end = min(n_act, (x + 1) * per);
    auto entry = [&](int r) { return x * per + r * nwg + ((r & 1) ? nwg - 1 - wg : wg); };
    // The source indices of each batch are loaded one batch ahead (the next
    // tile's first batch after a tile's last), so the visits hide that load.
    int idx = entry(0);
    int4 ent = idx < s_end ? sent[idx] : make_int4(0, 0, 0, 0);
    int pf = idx < s_end && ent.z + lane < ent.w ? src_idx[ent.z + lane] : 0;
    for (int r = 0; idx < s_end; ++r) {
        // (slot, tile, first source, end of sources) of this and the next tile
        const int nidx = entry(r + 1);
        const int4 nent = nidx < s_end ? sent[nidx] : make_int4(0, 0, 0, 0);
        const int a = ent.x;
        int lo[3];
        tile_coords(g, ent.y, lo);
        T acc[TILE][3];
#pragma unroll
        for (int xx = 0; xx < TILE; ++xx)
            acc[xx][0] = acc[xx][1] = acc[xx][2] = T(0);
        const int s0 = ent.z, s1 = ent.w;
        for (int sbat = s0; sbat < s1; sbat += 64) {
            const int sidx = sbat + lane;
            const int cur = pf;
            const bool more = sbat + 64 < s1;
            const int n0 = more ? sbat + 64 : nent.z, n1 = more ? s1 : nent.w;
            pf = n0 + lane < n1 ? src_idx[n0 + lane] : 0;
            int by = 64, bz = 64;       // no row for lanes past the list
            if (sidx < s1) {
                const int64_t i = cur;
                const typename Vec4<T>::type gq = s.geo[i];
                const typename Vec4<T>::type Fv = s.f4[i];
                int rb[3];
                unpack_rb(s.rb[i], rb);
                T gw[3][P];
                axis_weights_r<T, P>(gq.x, gw[0]);
                axis_weights_r<T, P>(gq.y, gw[1]);
                axis_weights_r<T, P>(gq.z, gw[2]);
                int b[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    int v = rb[ax] - lo[ax];
                    if (v < -(P - 1)) v += g.n[ax];
                    else if (v > TILE - 1) v -= g.n[ax];
                    b[ax] = v;
                }
                by = b[1];
                bz = b[2];
                // x weights: zeros, then the P weights at the stencil's offset
#pragma unroll
                for (int xx = 0; xx < TILE; ++xx)
                    sx[xx * 64 + lane] = T(0);
#pragma unroll
                for (int o = 0; o < P; ++o)
                    if ((unsigned)(b[0] + o) < (unsigned)TILE)
                        sx[(b[0] + o) * 64 + lane] = gw[0][o];
#pragma unroll
                for (int o = 0; o < P; ++o) {
                    sy[o * 64 + lane] = gw[1][o];
                    sz[o * 64 + lane] = gw[2][o];
                }
                sb[lane] = make_int2(lane - 64 * by, lane - 64 * bz);
                const T sc = use_dv ? gq.w : T(1);
                sf[0 * 64 + lane] = Fv.x * sc;
                sf[1 * 64 + lane] = Fv.y * sc;
                sf[2 * 64 + lane] = Fv.z * sc;
            }
            uint64_t my = 0, mz = 0;
#pragma unroll
            for (int k = 0; k < TILE; ++k) {
                const uint64_t yk = __ballot((unsigned)(k - by) < (unsigned)P);
                const uint64_t zk = __ballot((unsigned)(k - bz) < (unsigned)P);
                my = ly == k ? yk : my;
                mz = lz == k ? zk : mz;
            }
            __syncthreads();
            // Phase A: every lane visits up to K sources of its own row.
            // Phase B: what is left of the heavier rows is cut into pieces of
            // K sources dealt out to the lanes; the owners then add the
            // pieces in order.  K is the smallest cap whose pieces fit.
            uint64_t M = my & mz;
            const int n = __popcll(M);
            const int nmax = wave_max(n);
            // 64 K + MAXP K >= the batch's visits bounds K from below; the
            // cap rarely lies more than a few steps above that bound, so it
            // is searched upwards from there.
            int K = nmax;
            if (nmax > 1) {
                K = max(1, (wave_sum(n) + 63 + MAXP) / (64 + MAXP));
                while (K < nmax && wave_sum(n > K ? small_div(n - 1, K) : 0) > MAXP)
                    ++K;
            }
            for (int tt = 0; tt < K && M; ++tt) {
                const int k = __builtin_ctzll(M);
                M &= M - 1;
                visit(acc, ly, lz, k);
            }
            if (nmax > K) {
                const int np = n > K ? small_div(n - 1, K) : 0;   // pieces of this row
                const int ps = wave_exclusive_sum(np);
                rest[lane] = M;
                for (int q = 0; q < np; ++q)
                    piece[ps + q] = lane | (q << 8);
                const int NP = wave_sum(np);
                __syncthreads();
                T pacc[TILE][3];
#pragma unroll
                for (int xx = 0; xx < TILE; ++xx)
                    pacc[xx][0] = pacc[xx][1] = pacc[xx][2] = T(0);
                if (lane < NP) {
                    const int pr = piece[lane] & 255, pq = piece[lane] >> 8;
                    uint64_t m = drop_low_bits(rest[pr], pq * K);
                    for (int tt = 0; tt < K && m; ++tt) {
                        const int k = __builtin_ctzll(m);
                        m &= m - 1;
                        visit(pacc, pr & 7, pr >> 3, k);
                    }
                }
                __syncthreads();
                // the staged sources are no longer needed: pieces reuse them
                if (lane < NP) {
#pragma unroll
                    for (int xx = 0; xx < TILE; ++xx)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            buf[lane * 3 * TILE + 3 * xx + c] = pacc[xx][c];
                }
                __syncthreads();
                for (int q = 0; q < np; ++q) {
                    const T* pp = buf + (ps + q) * 3 * TILE;
#pragma unroll
                    for (int xx = 0; xx < TILE; ++xx)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            acc[xx][c] += pp[3 * xx + c];
                }
            }
            __syncthreads();
        }
        // the lane's row is 8 consecutive cells of each component in the slot;
        // with MASK, rows of zeros are not stored and their bit in the slot's
        // row mask (kept by slot and by tile) is clear
        bool nz = true;
        if constexpr (MASK) {
            nz = false;
#pragma unroll
            for (int xx = 0; xx < TILE; ++xx)
                nz = nz || acc[xx][0] != T(0) || acc[xx][1] != T(0) || acc[xx][2] != T(0);
            const uint64_t rm = __ballot(nz);
            if (lane == 0) {
                rmask[a] = rm;
                tmask[ent.y] = rm;
            }
        }
        T* gs = G + (int64_t)a * 3 * TILE_CELLS + TILE * lane;
        if (nz) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                typename Vec4<T>::type v0, v1;
                v0.x = acc[0][c];
                v0.y = acc[1][c];
                v0.z = acc[2][c];
                v0.w = acc[3][c];
                v1.x = acc[4][c];
                v1.y = acc[5][c];
                v1.z = acc[6][c];
                v1.w = acc[7][c];
                *reinterpret_cast<typename Vec4<T>::type*>(gs + c * TILE_CELLS) = v0;
                *reinterpret_cast<typename Vec4<T>::type*>(gs + c * TILE_CELLS + 4) = v1;
            }
        }
        idx = nidx;
        ent = nent;
    }
}

// The same spreading with one 2 x 2 x 2 block of the tile per lane instead
// of one row; it takes the entries of `sent` as k_spread_tiles does.
//
// Each lane holds one 2 x 2 x 2 block of the tile (lane = bx + 4 by + 16 bz,
// cells 2 bx .. 2 bx + 1 along x and so on).  Sources are staged 64 at a
// time as structure-of-arrays in LDS: per axis the P weights with a zero on
// each side, and F dV/h^3 (F alone when use_dv is 0: the transpose of
// interpolation in the adjoint).  Twelve ballots give, per block index along
// each axis, the 64-bit set of staged sources whose stencil overlaps it; a
// lane's own set is the AND of its three, and the lane visits exactly those
// sources in list order.  A stencil of P cells overlaps (P - 1)/2 + 1 blocks
// of 2 per axis on average, so a visit spends fewer of its multiply-adds on
// zero weights than a whole 8-cell row would, at the price of more work per
// visit (two dependent LDS reads, ten products besides the 24 multiply-adds)
// and a pass through LDS before the rows are stored.  It is the faster of the two for the 3-point kernel,
// whose stencil covers less of an 8-cell row; the rows are faster for the
// 4-point kernel.  A block cell just outside the stencil reads a zero pad.
// LDS stays near 6.5 KB so that 24 workgroups fit on a CU.
// (FP32: registers capped so that 6 waves fit per SIMD, the residency that the
// latency-bound visit chain wants.)
template <typename T, int P, bool MASK = false>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1, 8)))
k_spread_blocks(const int4* __restrict__ sent, const int32_t* __restrict__ nactive,
               const int32_t* __restrict__ src_idx, Grid g, MarkerData<T> s,
               T* __restrict__ G, uint64_t* __restrict__ rmask, uint64_t* __restrict__ tmask,
               int use_dv)
{
    constexpr int PW = P + 2;                              // weights per axis, zero padded
    constexpr int NW = 3 * PW + 3;                         // staged values per source
    constexpr int NBUF = NW * 64;
    constexpr int MAXP = NBUF / (3 * TILE) < 64 ? NBUF / (3 * TILE) : 64;   // phase-B pieces
    constexpr int NB = TILE / 2;                           // blocks per axis
    __shared__ __align__(16) T buf[NBUF];
    // per source k: o_a = k - 64 (b_a - 1) for the stencil base b_a along
    // axis a, so tile cell c's weight sits at s_a[64 c + o_a]; x and y in the
    // 16-bit halves of .x (|o_a| < 2^15), z in .y
    __shared__ int2 sb[64];
    T* const sx = buf;                  // [PW][64] zero, the P x weights, zero
    T* const sy = buf + PW * 64;        // [PW][64] y
    T* const sz = sy + PW * 64;         // [PW][64] z
    T* const sf = sz + PW * 64;         // [3][64]  F dV / h^3
    __shared__ uint64_t rest[64];       // sources of each block left after phase A
    __shared__ int32_t piece[MAXP];     // phase-B slot -> lane | piece << 8
    using T2 = typename Vec2<T>::type;
    // add source k's contribution to the 8 cells of block (cx, cy, cz):
    // a[z][y][x][c], with F wx and wy wz formed once per visit
    auto visit = [&](T (&a)[2][2][2][3], int cx, int cy, int cz, int k) {
        const int2 o = sb[k];
        const int ox = (int)(int16_t)(o.x & 0xffff), oy = o.x >> 16, oz = o.y;
        const T* px = sx + 128 * cx + ox;
        const T* py = sy + 128 * cy + oy;
        const T* pz = sz + 128 * cz + oz;
        const T wx[2] = {px[0], px[64]};
        const T wy0 = py[0], wy1 = py[64], wz0 = pz[0], wz1 = pz[64];
        const T f[3] = {sf[k], sf[64 + k], sf[128 + k]};
        const T t[2][2] = {{wy0 * wz0, wy1 * wz0}, {wy0 * wz1, wy1 * wz1}};   // [z][y]
#pragma unroll
        for (int xi = 0; xi < 2; ++xi) {
            const T u[3] = {f[0] * wx[xi], f[1] * wx[xi], f[2] * wx[xi]};
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        a[z][y][xi][c] += u[c] * t[z][y];
        }
    };
    const int lane = threadIdx.x;
    const int lbx = lane & 3, lby = (lane >> 2) & 3, lbz = lane >> 4;
    const int n_act = *nactive;
    const int per = (n_act + NXCD - 1) / NXCD;
    const int x = blockIdx.x % NXCD, nwg = gridDim.x / NXCD, wg = blockIdx.x / NXCD;
    const int s_end = min(n_act, (x + 1) * per);
    auto entry = [&](int r) { return x * per + r * nwg + ((r & 1) ? nwg - 1 - wg : wg); };
    // The source indices of each batch are loaded one batch ahead (the next
    // tile's first batch after a tile's last), so the visits hide that load.
    int idx = entry(0);
    int4 ent = idx < s_end ? sent[idx] : make_int4(0, 0, 0, 0);
    int pf = idx < s_end && ent.z + lane < ent.w ? src_idx[ent.z + lane] : 0;
    for (int r = 0; idx < s_end; ++r) {
        // (slot, tile, first source, end of sources) of this and the next tile
        const int nidx = entry(r + 1);
        const int4 nent = nidx < s_end ? sent[nidx] : make_int4(0, 0, 0, 0);
        const int a = ent.x;
        int lo[3];
        tile_coords(g, ent.y, lo);
        T acc[2][2][2][3];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx)
                    acc[z][y][xx][0] = acc[z][y][xx][1] = acc[z][y][xx][2] = T(0);
        const int s0 = ent.z, s1 = ent.w;
        for (int sbat = s0; sbat < s1; sbat += 64) {
            const int sidx = sbat + lane;
            const int cur = pf;
            const bool more = sbat + 64 < s1;
            const int n0 = more ? sbat + 64 : nent.z, n1 = more ? s1 : nent.w;
            pf = n0 + lane < n1 ? src_idx[n0 + lane] : 0;
            int b[3] = {64, 64, 64};    // no block for lanes past the list
            if (sidx < s1) {
                const int64_t i = cur;
                const typename Vec4<T>::type gq = s.geo[i];
                const typename Vec4<T>::type Fv = s.f4[i];
                int rb[3];
                unpack_rb(s.rb[i], rb);
                T gw[3][P];
                axis_weights_r<T, P>(gq.x, gw[0]);
                axis_weights_r<T, P>(gq.y, gw[1]);
                axis_weights_r<T, P>(gq.z, gw[2]);
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    int v = rb[ax] - lo[ax];
                    if (v < -(P - 1)) v += g.n[ax];
                    else if (v > TILE - 1) v -= g.n[ax];
                    b[ax] = v;
                }
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    T* sa = buf + ax * PW * 64;
                    sa[lane] = T(0);
#pragma unroll
                    for (int o = 0; o < P; ++o)
                        sa[(o + 1) * 64 + lane] = gw[ax][o];
                    sa[(P + 1) * 64 + lane] = T(0);
                }
                const int ox = lane - 64 * (b[0] - 1), oy = lane - 64 * (b[1] - 1);
                sb[lane] = make_int2((int)(((unsigned)ox & 0xffffu) | ((unsigned)oy << 16)),
                                     lane - 64 * (b[2] - 1));
                const T sc = use_dv ? gq.w : T(1);
                sf[0 * 64 + lane] = Fv.x * sc;
                sf[1 * 64 + lane] = Fv.y * sc;
                sf[2 * 64 + lane] = Fv.z * sc;
            }
            // block cb along an axis overlaps the stencil [b, b + P) when
            // b - 1 <= 2 cb <= b + P - 1
            uint64_t mx = 0, my = 0, mz = 0;
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const uint64_t xk = __ballot((unsigned)(2 * cb - b[0] + 1) < (unsigned)(P + 1));
                const uint64_t yk = __ballot((unsigned)(2 * cb - b[1] + 1) < (unsigned)(P + 1));
                const uint64_t zk = __ballot((unsigned)(2 * cb - b[2] + 1) < (unsigned)(P + 1));
                mx = lbx == cb ? xk : mx;
                my = lby == cb ? yk : my;
                mz = lbz == cb ? zk : mz;
            }
            __syncthreads();
            // Phase A: every lane visits up to K sources of its own block.
            // Phase B: what is left of the heavier blocks is cut into pieces
            // of K sources dealt out to the lanes; the owners then add the
            // pieces in order.  K is the smallest cap whose pieces fit.
            uint64_t M = mx & my & mz;
            const int n = __popcll(M);
            const int nmax = wave_max(n);
            // 64 K + MAXP K >= the batch's visits bounds K from below; the
            // cap rarely lies more than a few steps above that bound, so it
            // is searched upwards from there.
            int K = nmax;
            if (nmax > 1) {
                K = max(1, (wave_sum(n) + 63 + MAXP) / (64 + MAXP));
                while (K < nmax && wave_sum(n > K ? small_div(n - 1, K) : 0) > MAXP)
                    ++K;
            }
            for (int tt = 0; tt < K && M; ++tt) {
                const int k = __builtin_ctzll(M);
                M &= M - 1;
                visit(acc, lbx, lby, lbz, k);
            }
            if (nmax > K) {
                const int np = n > K ? small_div(n - 1, K) : 0;   // pieces of this block
                const int ps = wave_exclusive_sum(np);
                rest[lane] = M;
                for (int q = 0; q < np; ++q)
                    piece[ps + q] = lane | (q << 8);
                const int NP = wave_sum(np);
                __syncthreads();
                T pacc[2][2][2][3];
#pragma unroll
                for (int z = 0; z < 2; ++z)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int xx = 0; xx < 2; ++xx)
                            pacc[z][y][xx][0] = pacc[z][y][xx][1] = pacc[z][y][xx][2] = T(0);
                if (lane < NP) {
                    const int pr = piece[lane] & 255, pq = piece[lane] >> 8;
                    uint64_t m = drop_low_bits(rest[pr], pq * K);
                    for (int tt = 0; tt < K && m; ++tt) {
                        const int k = __builtin_ctzll(m);
                        m &= m - 1;
                        visit(pacc, pr & 3, (pr >> 2) & 3, pr >> 4, k);
                    }
                }
                __syncthreads();
                // the staged sources are no longer needed: pieces reuse them
                if (lane < NP) {
                    T* pp = buf + lane * 3 * TILE;
#pragma unroll
                    for (int z = 0; z < 2; ++z)
#pragma unroll
                        for (int y = 0; y < 2; ++y)
#pragma unroll
                            for (int xx = 0; xx < 2; ++xx)
#pragma unroll
                                for (int c = 0; c < 3; ++c)
                                    pp[((z * 2 + y) * 2 + xx) * 3 + c] = pacc[z][y][xx][c];
                }
                __syncthreads();
                for (int q = 0; q < np; ++q) {
                    const T* pp = buf + (ps + q) * 3 * TILE;
#pragma unroll
                    for (int z = 0; z < 2; ++z)
#pragma unroll
                        for (int y = 0; y < 2; ++y)
#pragma unroll
                            for (int xx = 0; xx < 2; ++xx)
#pragma unroll
                                for (int c = 0; c < 3; ++c)
                                    acc[z][y][xx][c] += pp[((z * 2 + y) * 2 + xx) * 3 + c];
                }
            }
            __syncthreads();
        }
        // the block goes to the slot through LDS, one component at a time,
        // so that each lane stores one whole row (8 cells, contiguous in the
        // slot) as the row layout does; with MASK, rows of zeros are not
        // stored and their bit in the slot's row mask (kept by slot and by
        // tile) is clear: row (y, z) is bit y + 8 z, held by the four lanes
        // of its blocks along x
        bool row_nz = true;
        if constexpr (MASK) {
            uint64_t bl[2][2];
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    bool v = false;
#pragma unroll
                    for (int xx = 0; xx < 2; ++xx)
                        v = v || acc[z][y][xx][0] != T(0) || acc[z][y][xx][1] != T(0) ||
                            acc[z][y][xx][2] != T(0);
                    bl[z][y] = __ballot(v);
                }
            // lane j decides row j: y = j & 7, z = j >> 3
            const int ry = lane & 7, rz = lane >> 3;
            const uint64_t sel = (rz & 1) ? ((ry & 1) ? bl[1][1] : bl[1][0])
                                          : ((ry & 1) ? bl[0][1] : bl[0][0]);
            row_nz = ((sel >> (4 * (ry >> 1) + 16 * (rz >> 1))) & 0xfull) != 0;
            const uint64_t rm = __ballot(row_nz);
            if (lane == 0) {
                rmask[a] = rm;
                tmask[ent.y] = rm;
            }
        }
        static_assert(TILE_CELLS <= NBUF, "one component of the tile fits the staging buffer");
        T* gs = G + (int64_t)a * 3 * TILE_CELLS + TILE * lane;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    T2 v;
                    v.x = acc[z][y][0][c];
                    v.y = acc[z][y][1][c];
                    *reinterpret_cast<T2*>(buf + TILE * TILE * (2 * lbz + z) +
                                           TILE * (2 * lby + y) + 2 * lbx) = v;
                }
            __syncthreads();
            const typename Vec4<T>::type v0 =
                *reinterpret_cast<const typename Vec4<T>::type*>(buf + TILE * lane);
            const typename Vec4<T>::type v1 =
                *reinterpret_cast<const typename Vec4<T>::type*>(buf + TILE * lane + 4);
            __syncthreads();
            if (row_nz) {
                *reinterpret_cast<typename Vec4<T>::type*>(gs + c * TILE_CELLS) = v0;
                *reinterpret_cast<typename Vec4<T>::type*>(gs + c * TILE_CELLS + 4) = v1;
            }
        }
        idx = nidx;
        ent = nent;
    }
}
