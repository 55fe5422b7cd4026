// paths.h -- host-side entry points of the plain and batched loops.
#pragma once

#include "ibx_internal.h"

namespace ibx {

void desired_velocity(const ib_particles* p, const ib_markers* m, ib_prec prec, void* Ud,
                      hipStream_t st);

// Deterministic sum (fixed chunking and tree) of v[0..n) into *out (sqrt if asked).
void sum_to(const double* v, int64_t n, double* part, double* out, bool do_sqrt, hipStream_t st);
size_t sum_partials(int64_t n);
size_t field_elems(const Grid& g);

void plain_interp(const Grid& g, int P, ib_prec prec, const ib_markers* m, const void* u,
                  void* U, hipStream_t st);
void plain_spread(const Grid& g, int P, ib_prec prec, const ib_markers* m, const ib_buckets* b,
                  const void* F, void* f, double scale, int use_dv, hipStream_t st);

size_t plain_workspace(const Grid& g, ib_prec prec, int64_t nl);
int plain_multidirect(const Grid& g, int P, ib_prec prec, const ib_particles* p,
                      const ib_markers* m, const ib_buckets* b, int ns, double dt,
                      const void* u0, void* ustar, void* f, void* F, double* resid, void* Fhist,
                      void* ws, size_t ws_bytes, hipStream_t st);

struct BatchedCfg {
    int bw;        // markers per interpolation work item (= threads per workgroup)
    int ncu;       // compute units of the device
    int wgs_s;     // cap on resident spreading workgroups per CU (0 = as many as fit)
    int masks;     // G slot row masks: zero rows neither stored nor loaded
    int txw;       // x extent of an interpolation work tile: 8 (one tile) or 16 (FP32)
    Profiler* prof;  // nullable: per-kernel event timing
};

size_t batched_workspace(const Grid& g, ib_prec prec, int64_t nl, const BatchedCfg& cfg);
int batched_multidirect(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                        const ib_particles* p, const ib_markers* m, const ib_buckets* b, int ns,
                        double dt, const void* u0, void* ustar, void* f, void* F, double* resid,
                        void* Fhist, void* ws, size_t ws_bytes, hipStream_t st, int f_acc = 0);

// Spreading with the loop's tile kernel outside the loop (the adjoint):
// records and work lists once per call, then out = S v (use_dv: with dV/h^3,
// else without) on every valid covered cell, or out = u0 + dt S v when u0 is
// given.  v: [nl][3] in marker order.  Grids with fewer than 16 cells on an
// axis, or boxes above 512, are not supported (tile_spread_supported).
bool tile_spread_supported(const Grid& g);
size_t tile_spread_workspace(const Grid& g, ib_prec prec, int64_t nl);
int tile_spread_setup(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                      const ib_particles* p, const ib_markers* m, const ib_buckets* b, void* ws,
                      size_t ws_bytes, hipStream_t st);
int tile_spread(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg, const ib_markers* m,
                const ib_buckets* b, const void* v, int use_dv, const void* u0, double dt,
                void* out, void* ws, size_t ws_bytes, hipStream_t st);
// With the same set-up: U = J fld (U nullable, marker order) and
// gX += sc sum over the stencil of (fld . v_l) grad_X w_l, sc = dV/h^3
// (use_dv) or 1, for a field fld in the box layout and v [nl][3].
int tile_interp_grad(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                     const ib_markers* m, const ib_buckets* b, const void* fld, const void* v,
                     void* U, int use_dv, double* gX, void* ws, size_t ws_bytes, hipStream_t st);

// Particle-by-particle order of the loop, run level by level (sequential.hip).
constexpr int SEQ_MAX_LEVELS = 4096;
size_t sequential_workspace(const ib_level* lv, const Grid& g, ib_prec prec, int32_t np,
                            int64_t nl, const BatchedCfg& cfg);
int sequential_multidirect(const ib_level* lv, const Grid& g, int P, ib_prec prec,
                           const BatchedCfg& cfg, const ib_particles* p, const ib_markers* m,
                           int ns, double dt, const int32_t* level, int32_t nlevels,
                           const void* u0, void* ustar, void* f, void* F, int32_t* flag,
                           void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace ibx

namespace ibx {
size_t backward_workspace(const Grid& g, ib_prec prec, int64_t nl);
int multidirect_backward(const Grid& g, int P, ib_prec prec, const BatchedCfg& cfg,
                         const ib_particles* p,
                         const ib_markers* m, const ib_buckets* b, int ns, double dt,
                         const void* u0, const void* Fhist, const void* gus, const void* gf,
                         const void* gF, void* gu0, double* gup, double* gom, double* gX,
                         void* ws, size_t ws_bytes, hipStream_t st);
}  // namespace ibx
