// lbm_internal.hpp -- launchers shared between the ABI (lbm_abi.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.hpp"

namespace lbm {

constexpr int kTileX = 256;      // nodes (work-items) per work-group of the step kernel
constexpr int kObserveWG = 512;  // work-groups of the observables pass
constexpr int kObsParts = 6;     // partial results per work-group of the observables pass
constexpr int kObsOut = 2 + kObsParts;  // results of the observables pass (Nu_hot, Nu_cold, ...)
constexpr int kPitchAlign = 64;  // row pitch in elements
// Elements between the end of one plane's rows and the start of the next (4 KiB + 128 B in
// FP32).  Without it the planes of a 4096-wide power-of-two grid lie exactly 64 MiB apart and
// the 14 + 2 streams of a row fall on the same memory channel and bank; with it the two-step
// kernel on the 4096^2 workload ran 1-2 % faster (71.5k against 69.5k-70.7k MLUPS, with the
// same fetched bytes).  A stride of +64 or +4160 elements measured within 0.5 % of this one.
constexpr int kPlanePad = 1056;

// Elements per plane: ny rows of the pitch, then the pad.
inline long long plane_elems(long long pitch, long long ny) { return pitch * ny + kPlanePad; }

// Two steps per launch: columns a wavefront's strip writes, strips per work-group, the number
// of resident-set rounds the segment height aims for, and the shortest segment.
constexpr int kTbCols = 62;
constexpr int kTbWaves = 4;
constexpr int kTbRounds = 12;
constexpr int kTbMinRows = 6;
// The shortest segment the batch's autotuner tries.
constexpr int kBatchTbMinRows = 2;
// Minimum wavefronts per SIMD the two-step kernels are compiled for: in FP32 four, the
// occupancy their ~128 registers allow (the compiler would otherwise settle for 129 registers
// and three); the FP64-arithmetic forms take what their registers give.
template <typename S, typename R>
constexpr int tb_min_waves() {
    return sizeof(S) == 4 && sizeof(R) == 4 ? 4 : 1;
}

// Several steps per launch on small grids (lbm_tile.hip), in two forms of the same region
// (a tile, a halo as wide as the steps, and one node more at a wall: 25 x 25 nodes at most):
// 16 x 16 tiles advanced four steps, and on the smallest grids 8 x 8 tiles advanced eight.
constexpr int kTileSide = 16;
constexpr int kTileSteps = 4;
constexpr int kTinyTileSide = 8;
constexpr int kTinyTileSteps = 8;
constexpr int kTileThreads = 640;   // one work-item per node of the largest region (25^2)
static_assert(kTileSide + 2 * kTileSteps == kTinyTileSide + 2 * kTinyTileSteps,
              "both tile forms share one region size");
// Tile side of the form that takes k steps per launch
constexpr int tile_side(int k) { return k == kTinyTileSteps ? kTinyTileSide : kTileSide; }

// The two-step kernels address a state (the 14 planes) through raw buffer descriptors and drop
// stores through an offset of 2^31 past them, so a descriptor covers less than 2^31 bytes: one
// descriptor for a state below 2^31 bytes, two (planes 0-6 and 7-13) for a state whose halves
// are.  tb2_descs gives the number of descriptors a state needs, 0 if even its halves are too
// large.  The batched two-step kernel uses one descriptor per cavity.
inline int tb2_descs(const Geo& G, size_t elem_bytes) {
    const unsigned long long pb = (unsigned long long)G.plane * elem_bytes;
    if (kPlanes * pb < (1ull << 31)) return 1;
    if (kPlanes / 2 * pb < (1ull << 31)) return 2;
    return 0;
}
inline bool tb2_fits(const Geo& G, size_t elem_bytes) { return tb2_descs(G, elem_bytes) > 0; }

// Launchers take S, the storage type of populations and medium planes, and R, the arithmetic
// type; instantiated for (float, float), (double, double) and (float, double).

template <typename S, typename R>
hipError_t launch_step(const void* src, void* dst, const void* med, const Geo& G,
                       const Phys<R>& P, hipStream_t s);
// Queries the device once for the two-step kernel's launch shape (call outside graph capture)
template <typename S, typename R>
void prepare_tb2();
// Whether two steps per launch are faster than one for this grid and these types
template <typename S, typename R>
bool tb2_pays(const Geo& G, bool per_node_medium);
// Steps per launch of the tile form that is fastest for this grid and these types, if one beats
// a step per launch (kTileSteps or kTinyTileSteps), else 0
template <typename S, typename R>
int tile_steps(const Geo& G, bool per_node_medium);
// k (kTileSteps or kTinyTileSteps) steps of the pull layout from src to dst, each tile of the
// grid advanced in LDS
template <typename S, typename R>
hipError_t launch_tile_step(const void* src, void* dst, const void* med, const Geo& G,
                            const Phys<R>& P, int k, hipStream_t s);
// Three steps per launch (FP32 storage and arithmetic only; hipErrorInvalidValue otherwise, or
// for a state of 2 GiB or more): whether they are faster than two for this grid; rows per
// segment, segments and work-groups per launch; the launch, src (step n) to dst (step n + 3)
template <typename S, typename R>
bool tb3_pays(const Geo& G, bool per_node_medium);
template <typename S, typename R>
void tb3_shape(const Geo& G, bool per_node_medium, int* rows, int* nseg, int* nwg);
template <typename S, typename R>
hipError_t launch_tb3_step(const void* src, void* dst, const void* med, const Geo& G,
                           const Phys<R>& P, hipStream_t s);
// Rows per segment and work-groups per launch of the two-step kernel
template <typename S, typename R>
void tb2_shape(const Geo& G, bool per_node_medium, int* rows, int* nwg);
// Two pull-layout steps in one launch, src (step n) to dst (step n + 2)
template <typename S, typename R>
hipError_t launch_tb2_step(const void* src, void* dst, const void* med, const Geo& G,
                           const Phys<R>& P, hipStream_t s);
// AA-pattern step in place; parity 0: the state is in the kAAOpp form, 1: kAAOwn
template <typename S, typename R>
hipError_t launch_aa_step(void* buf, const void* med, const Geo& G, const Phys<R>& P,
                          int parity, hipStream_t s);
// layout: the PopLayout form the state is in
template <typename S, typename R>
hipError_t launch_observe(const void* src, const void* med, const Geo& G, const Phys<R>& P,
                          int layout, void* ux, void* uy, void* p, void* T, double* part,
                          int nparts, double L_over_dT, double* out, hipStream_t s);
template <typename S, typename R>
hipError_t launch_stream_function(const void* src, const void* med, const Geo& G,
                                  const Phys<R>& P, int layout, void* psi, hipStream_t s);
template <typename R>
hipError_t launch_rest(void* dst, const Geo& G, double g0, double g1, hipStream_t s);
template <typename R>
hipError_t launch_pitch_copy(void* dst, const void* src, const Geo& G, double v, hipStream_t s);

// Adjoint (lbm_adjoint.hip)
template <typename S, typename R>
hipError_t launch_adjoint_seed(const void* state, void* lam, const Geo& G, const Phys<R>& P,
                               double L_over_dT, hipStream_t s);
template <typename S, typename R>
hipError_t launch_adjoint_step(const void* state, const void* lam_in, void* lam_out,
                               const void* med, double* gphi, double* gK, const Geo& G,
                               const Phys<R>& P, hipStream_t s);
template <typename R>
hipError_t launch_fill(void* dst, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double* dst, size_t n, hipStream_t s);
hipError_t launch_unpitch_scale(double* dst, const double* src, const Geo& G, double scale,
                                hipStream_t s);

// Batched form (lbm_batch.hip)
struct BatchCavity {
    Geo G;
    long long off;     // element offset of the cavity's state inside a state buffer
    int tile0;         // first tile id of the cavity
    int tiles_x;       // tiles along x
};

template <typename R>
struct BatchTable {
    const BatchCavity* cav;  // device array [n]
    const Phys<R>* phys;     // device array [n]
    const int* tile_cav;     // device array [ntiles]: cavity of each tile
    int ncav;
    int ntiles;
};

// Two steps per launch for every cavity of a batch: T.tile_cav maps each logical work-group to
// its cavity, whose tile0 is its first work-group and tiles_x its number of strip groups (of
// `waves` strips: 1, 2 or 4); rows: rows per segment.
template <typename S, typename R>
hipError_t launch_batch_tb2(const void* src, void* dst, const BatchTable<R>& T, int rows,
                            int waves, hipStream_t s);
// Queries the batched two-step kernel's resident set once (call outside graph capture)
template <typename S, typename R>
void prepare_batch_tb2();

// rows: rows per tile (work-group = 64 * rows work-items); nodes_x: 64-node segments per
// work-item along x; nwg >= ntiles: one tile per work-group, else chunked persistent.
template <typename S, typename R>
hipError_t launch_batch_step(const void* src, void* dst, const BatchTable<R>& T, int nodes_x,
                             int rows, int nwg, hipStream_t s);

}  // namespace lbm
