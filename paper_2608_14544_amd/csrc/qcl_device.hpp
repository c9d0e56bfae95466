// Device-side structures and constants shared by the library's kernels and
// by the kernels compiled at run time for models with a supplied potential.
// Kept free of host-only headers; the constants come from the public header
// (QCL_TILE, QCL_FLAG_*, QCL_MAX_MODES), which the includer has seen, or
// from definitions the run-time compilation puts in front.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

namespace qcl {

constexpr int kBlock = QCL_TILE;           // walkers per workgroup == reduction tile
constexpr int kWave = 64;                  // CDNA wavefront
constexpr int kMaxFastModes = 8;           // N = 2 kernels specialised on M = 1..8

// Per-walker flag bits (mirrors the public QCL_FLAG_* values).
constexpr uint32_t kFlagNonfinite = QCL_FLAG_NONFINITE;
constexpr uint32_t kFlagDegenerate = QCL_FLAG_DEGENERATE;
constexpr uint32_t kFlagResolved = QCL_FLAG_RESOLVED64;
constexpr uint32_t kFlagFallback = QCL_FLAG_FALLBACK;

template <typename R>
struct EnsDev {
    R *q;
    R *p;
    R *u;
    double *w;
    double *phase;
    uint8_t *a;
    uint8_t *b;
    uint32_t *flags;
    int64_t ld;
    int64_t n_traj;
    int64_t traj_offset;
};

struct SampleArgs {
    double q0[QCL_MAX_MODES];
    double sq[QCL_MAX_MODES];
    double sp[QCL_MAX_MODES];
    int32_t state;
    int32_t basis;
    uint32_t key0, key1;
    int32_t m;  // modes actually present (general kernels)
};

struct PropArgs {
    int64_t step0;
    int32_t n_steps;
    int32_t cadence;
    int32_t n_out;
    int32_t scheme;
    uint32_t key0, key1;
    int32_t m;  // modes actually present (general kernels)
};

// Step constants of a model with a supplied potential (binary64)
struct UserArgs {
    double dt, hdt;
    double dt_hbar;
    double rot_eps;  // Jacobi: rotate while |a_pq| > rot_eps * ||A||_F
    double gap_thr;  // binary32 step: gaps below this are re-solved in binary64
};

// One (instance, tile) work item of a batched call for a model with a
// supplied potential: the same layout on the host, which writes it, and in
// the run-time compiled kernel, which reads it
template <typename R>
struct UserBatchItem {
    UserArgs A;
    PropArgs P;
    EnsDev<R> E;
    double *partials;
    int64_t tile_begin;
};
static_assert(sizeof(PropArgs) == 40 && sizeof(EnsDev<double>) == 88 && sizeof(UserBatchItem<double>) == 184 &&
                  sizeof(UserBatchItem<float>) == 184,
              "the batch descriptor must have one layout on the host and in the compiled program");

// One bin of one tile's partials: the 8 N^2 sums [2][N][N][Re, Im, Re^2,
// Im^2], then the number of walkers excluded from the bin (non-finite weight
// or phase), stored as a double so that the tile reduction adds it exactly.
__host__ __device__ constexpr int64_t tile_values(int n_states) { return 8LL * n_states * n_states + 1; }

}  // namespace qcl
