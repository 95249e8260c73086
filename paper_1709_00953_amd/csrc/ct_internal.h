// Internal structures shared by the host runtime (ct_api.cpp) and the gfx950
// kernels (ct_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {

constexpr int kChunk = 64;         // rays per forward chunk (one wave's lanes)
constexpr int kSplit = 4;          // waves per forward work-group; each walks 1/kSplit of every chord
constexpr int kMaxInline = 128;    // row blocks passed by value to a primitive launch
constexpr int kTile2 = 8;          // 2D back-projection tile: 8 x 8 voxels, 4 waves split the views
constexpr int kTile3x = 8, kTile3y = 8, kTile3z = 4;   // 3D tile: 8 x 8 x 4
// Per-view float64 frame: a(3) c(3) e_u(3) e_v(3) n(3) sdd|kappa, 1/sdd, sigma.
constexpr int kViewStride = 24;
// A unit ray direction component at most this large is taken as exactly zero:
// it is float64 residue of an axis-parallel ray (cos of a quarter turn is
// 6e-17), a tilt the float32 slab clip cannot resolve (its slab interval
// endpoints would cancel), while the exact-zero half-open membership test can.
constexpr double kAxisEps = 1e-12;
constexpr float kAxisEpsF = 1e-12f;
// 3D back-projection: views whose detector window holds a ray with a direction
// component (in units of the ray vector over the source-detector distance)
// below this take the float64 candidate path (clip3_precise)
constexpr double kNearAxis = 0.02;
enum { kPar2D = 0, kFanFlat = 1, kFanCurved = 2, kCone = 3 };
// Launch kind of a cone geometry whose every view has its detector columns
// parallel to the z axis (e_v = +-z, e_u and the source-detector axis in the
// xy plane): its back-projection takes the voxel-column kernel.
constexpr int kConeV = 4;

// Voxel-column tile of that kernel: CX x CY columns of TZ voxels in z, 256
// lanes, each lane VZ voxels of a column (levels l, l + TZ / VZ, ...): eight,
// or TZ when TZ < 8.  More voxels a lane share its per-view work (the window's
// staging, the view's constants) among more voxels: on the 256^3 cone's
// back-projection, 2.80 ms per launch with two, 2.18 with four; after the
// voxel path's later cuts 1.89 with four and 1.85 with eight (119 registers,
// four work-groups per CU).  TZ is the largest power of two up to 32 whose
// tiles waste at most 1/8 of the voxels over the box's nz (at least 1).
constexpr int kColVoxels = 8;       // voxels a lane at most
__host__ __device__ inline int col_vz(int tz) { return tz >= 8 ? 8 : tz; }
__host__ __device__ inline void col_tile_shape(int nz, int& tz, int& cx, int& cy) {
    int t = 32;
    while (t > 1 && ((nz + t - 1) / t) * t - nz > nz / 8) t >>= 1;
    tz = t;
    const int nc = 256 / (t / col_vz(t));    // 64 .. 256 columns
    int lg = 0;
    while ((1 << lg) < nc) ++lg;
    cx = 1 << ((lg + 1) / 2);
    cy = nc / cx;
}

// J-local (x, g) pairs of a group are stored twice: copy 0 x-fastest
// ([z][y][x]) and copy 1 y-fastest ([z][x][y]).  The forward pass reads the
// copy whose fast axis runs across its rays, so the lanes of a wave (adjacent
// rays) gather adjacent pixels.  The walk forms kWalkU segments before their
// gathers, so it can step past the box by one crossing that float32 rounding
// places before the exit, then by up to kWalkU - 1 more to the end of the
// batch, each by at most the largest index stride.  The 2D slab walk runs at
// most kWalkU - 1 slab rows past the box (one row stride each) and reads a
// pair that starts one element before a row or ends one element after it.
// Each copy has xg_pad zero elements before and after it, enough for those
// steps and one more: they read finite values for segments of zero length,
// with no bounds check.  Where column blocks differ in size, the step's
// finalize clears the copies after reading them: a block of another size
// lays its copies out differently, so this step's pairs could otherwise lie
// in the padding of a later step's.
constexpr int kWalkU = 4;
__host__ __device__ inline int xg_pad(int nx, int ny, int nz) {
    const int step = nz > 1 ? nx * ny : (nx > ny ? nx : ny);
    return (kWalkU + 1) * step + 64;
}
__host__ __device__ inline int xg_copy(int nx, int ny, int nz) { return nx * ny * nz + 2 * xg_pad(nx, ny, nz); }
__host__ __device__ inline int xg_size(int nx, int ny, int nz) { return 2 * xg_copy(nx, ny, nz); }

// One detector tile of a row block: rays (view, v0..v1-1, u0..u1-1).
struct Tile {
    int32_t view, u0, u1, v0, v1;
};

// Up to kChunk consecutive rays of a detector rectangle of one view
// (v-major, u fastest): ray k of the rectangle is (v0 + k / w, u0 + k % w).
// The rectangle is a whole tile (row-block chunk lists) or the part of a
// tile whose rays can meet one column block (windowed lists).
struct Chunk {
    int32_t view, u0, v0, w;
    int32_t k0;     // first ray within the rectangle
    int32_t cnt;    // rays in the chunk
    int32_t roff;   // offset of the first ray within its (windowed) row block
    int32_t pad;
};

// A row block taking part in a launch.  chunk_prefix / slot_prefix are the
// numbers of chunks / rays of the launch that precede this entry.
struct Entry {
    int32_t rb;
    int32_t group;          // group index within the launch (0 for primitives)
    int32_t chunk_prefix;
    int32_t slot_prefix;
};

// Per-(view, bin) data of a 2D ray, built on the host in float64.
// Forward: unit direction (dx, dy) and its reciprocals (0 where a component is
// exactly zero).
struct Ray2F {
    double dx, dy, idx, idy;
};
// Back-projection: delta = p*B - q*A is the signed distance of the ray from a
// voxel centre whose view-frame coordinates are (A, B).  For a unit direction
// (dx, dy) with both components nonzero the clip length with a voxel of
// half-widths (hx, hy) is the trapezoid
//   clamp((hs - |delta|) K, 0, M),  hs = hx |dy| + hy |dx|,  K = 1 / |dx dy|,
//   M = min(2 hx / |dx|, 2 hy / |dy|).
// hs - |delta| is formed in float64: for a ray nearly parallel to an axis K is
// large, and the difference is the small distance of the ray from the voxel's
// corner band, which float32 operands ~hs (relative error 6e-8) would swamp.
// A zero direction component is marked by M = -1 (dx = 0) or M = -2 (dy = 0);
// then K is the full chord and hs the index of the one x (or y) slab the ray
// lies in.
struct Ray2B {
    double p, q, hs;
    float K, M;
};
// The curved fan's float32 form of the same clip, for rays with
// min(|dx|, |dy|) >= 0.02 only: (K, S = hs K, M, 0).
struct Ray2K {
    float K, S, M, pad;
};

// Device-side geometry, passed by value.
struct DGeom {
    int32_t kind, nx, ny, nz, nu, nv, n_views;
    int32_t dims;
    double vx, vy, vz, ox, oy, oz, pu, pv;
    double ivx, ivy, ivz;         // reciprocal voxel pitch
    float radius;                 // voxel half-diagonal (mm)
    const double* view64;         // [n_views][kViewStride]
    const Ray2F* ray2f;           // [n_views][nu] (2D kinds)
    const Ray2B* ray2b;           // [n_views][nu] (2D kinds)
    const Ray2K* ray2k;           // [n_views][nu] (curved fan)
    // vertical cones (kConeV): float32 components D~_x, D~_y of the rays of
    // each detector column (the values every cone kernel forms,
    // (float)(D_k / sdd)) with D~_x^2 + D~_y^2 (from float64) and a zero, D~_z
    // of each row, and 2^colk_e sdd / D_z of each row in float64 (0 for a
    // zero component)
    const float4* cdxy;           // [n_views][nu]
    const float* cdz;             // [n_views][nv]
    const double* cisv;           // [n_views][nv]
    const int32_t* view_flags;    // [n_views] bit0: some ray has a zero direction component
    const Tile* tiles;
    const int32_t* rb_tile_ptr;
    const int32_t* tile_roff;     // first ray of the tile within its row block
    const Chunk* chunks;           // whole row blocks
    const int32_t* rb_chunk_ptr;  // [m+1]
    const Chunk* wchunks;         // row block x column block windows
    const int32_t* rbj_chunk_ptr; // [m*n+1], index rb*n + J
    int32_t n_cols;
    int32_t mixed_boxes;          // column blocks differ in size (their (x, g) copies differ in layout)
    int32_t vertical;             // cone: every view's detector columns run along z (kConeV)
    // vertical cones: the exponent e of 2^e, the largest power of two at most
    // 1 / (the xy diagonal of a voxel).  A ray's parameter s (point =
    // S + s D / sdd) spans at most that diagonal in a voxel column, as
    // |D_xy| >= sdd, so every clip length times 2^e is at most 1; the scaling
    // is exact.  The table cisv holds 2^e sdd / D_z.
    int32_t colk_e;
};

struct Box {
    int32_t x0, x1, y0, y1, z0, z1;
};

// Forward launch: rays of the entries' row blocks through box J.
struct FwdCore {
    static constexpr bool kInl = false;
    Box box;
    const Entry* ent;             // entries (device); FwdArgs may pass them inline instead
    int32_t n_ent;
    int32_t n_chunks;
    int32_t flags;                // CT_ACCUMULATE
    int32_t mode;                 // 0 single, 1 fused (x,g), 2 count
    int32_t windowed;             // 1: chunks of the (row block, col) windows
    const float* x;               // single: full volume
    const float2* xg;             // fused: [group][xg_stride] (x_J, g_J), two J-local copies
    int32_t vox_J;                // |J|
    int32_t xg_stride;            // per-group stride of xg (both padded copies)
    float* out;                   // single/fused: ray-indexed (Ax)
    float* q;                     // fused: slot-indexed A g
    double* partial;              // fused: per chunk sum (A g)^2
    unsigned long long* nnz;      // count: [m][n]
    int32_t n_cols, col;          // count: column count and this column
    double tau;                   // count threshold
    int32_t split = kSplit;       // fused: pieces per chord (waves per 64 rays): 1, 2 or 4
};
struct FwdArgs : FwdCore {
    static constexpr bool kInl = true;
    Entry inl[kMaxInline];        // used when ent is nullptr
};

// Back-projection launch: group g's row blocks are entries [gptr[g], gptr[g+1]).
struct BackCore {
    static constexpr bool kInl = false;
    Box box;
    const Entry* ent;
    const int32_t* gptr;          // device or nullptr (single group of all entries)
    int32_t n_ent;
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t flags;
    int32_t fused;                // 1: write (x_J, g_J) float2 + partial
    const float* r;               // ray-indexed
    const float* x;               // full volume (fused: copied into xg)
    float* g;                     // single: full volume
    float2* xg;                   // fused: [group][xg_stride], two J-local copies
    int32_t vox_J;
    int32_t xg_stride;
    double* partial;              // fused: [group][tiles]
};
struct BackArgs : BackCore {
    static constexpr bool kInl = true;
    Entry inl[kMaxInline];
};

// Finalize of one column-block step (ray part, then voxel part).
// Step sizes of one column-block step: group g's ||g||^2 partials are
// pg[g*n_tiles ..], its ||A g||^2 partials those of its entries' chunks.
struct StepArgs {
    const Entry* ent;
    const int32_t* gptr;    // group -> entries
    int32_t n_chunks;
    int32_t n_tiles;        // back-projection tiles per group
    const double* pg;
    const double* pq;
    const double* beta;     // [G]
    double* mu;             // [G]
};

struct FinArgs {
    static constexpr bool kInl = false;
    const Entry* ent;
    int32_t n_ent;
    int32_t n_chunks;
    const double* mu;       // [G]
    const float* q;
    float* z;               // [n][M]
    float* zJ;              // z + J*M
    const float* y;
    float* r;
    int64_t M;
    int32_t n_cols;
    int32_t refresh;        // 1: r = y - sum_j z^j on the step's rays
    int32_t col;            // column block (windowed chunk lists)
    // voxel part
    Box box;
    int32_t vox_J;
    int32_t xg_stride;
    int32_t n_groups;
    float2* xg;             // read; cleared after the read where column blocks differ in size
    float* x;
    int32_t nx, ny;
};

// Residual refresh over the rays of a list of row blocks.
struct ResArgs {
    static constexpr bool kInl = false;
    const Entry* ent;
    int32_t n_ent;
    const float* z;
    const float* y;
    float* r;
    int64_t M;
    int32_t n_cols;
};

// ---------------------------------------------------------------------------
// batches: several independent jobs advanced by the same launches
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 256;     // jobs in one batch

// One column-block step of a schedule as the batched kernels read it.
struct StepRec {
    int32_t col;        // column block J
    int32_t n_groups;
    int32_t ent_off;    // the step's entries: ent[ent_off, ent_off + n_ent)
    int32_t n_ent;
    int32_t gptr_off;   // group -> entry offsets: gptr[gptr_off, gptr_off + n_groups]
    int32_t beta_off;   // beta[beta_off, beta_off + n_groups)
    int32_t n_chunks;   // windowed chunks of the step
    int32_t pad;
};

struct EpochRec {
    int32_t step0, n_steps;              // steps[step0, step0 + n_steps)
    int32_t uni_off, n_uni, uni_chunks;  // row blocks touched in the epoch
    int32_t pad;
};

// A job of a batch: geometry, solver buffers, data and schedule, all device
// pointers.  The job's next epoch is the batch's counter ep[k].
struct BJob {
    DGeom G;
    const Box* boxes;             // [n_cols]
    float* z;
    float* r;
    float* q;
    float2* xg;
    double* pg;
    double* pq;
    double* mu;
    const float* y;
    float* x;
    const StepRec* steps;
    const EpochRec* epochs;
    const Entry* ent;
    const int32_t* gptr;
    const double* beta;
    const Entry* uni;
    int64_t M;
    int32_t n_epochs;
    int32_t sync;                 // 0 column, 1 epoch
    int32_t kind;
    int32_t pad;
};

// One phase of one step index for every job of a batch.  Work-group b
// belongs to the job k with prefix[k] <= b < prefix[k + 1] (local index
// b - prefix[k]); jobs whose current epoch has no such step, or that have
// run all their epochs, return at once.
struct BatchArgs {
    const BJob* jobs;
    int32_t* ep;                  // per-job next epoch
    const int32_t* prefix;        // [n_jobs + 1]
    int32_t n_jobs;
    int32_t c;                    // step index within the epoch
};

enum { kPhBack = 0, kPhFwd = 1, kPhStep = 2, kPhFin = 3, kPhRes = 4 };

// Records a message for ct_last_error() and returns code.
int fail(int code, const char* fmt, ...);

hipError_t launch_fwd(const DGeom& G, const FwdArgs& a, hipStream_t st);
// Launch-shape choices of the projectors (picked by the tuner, or set):
// pieces per chord of the fused forward and waves per 2D back-projection tile.
struct Tune {
    int32_t split = kSplit;
    int32_t waves = 4;
};
hipError_t launch_back(const DGeom& G, const BackArgs& a, int n_groups, int waves, hipStream_t st);
hipError_t launch_step(const StepArgs& s, int n_groups, hipStream_t st);
hipError_t launch_finalize(const DGeom& G, const FinArgs& f, int vox_blocks, hipStream_t st);
hipError_t launch_residual(const DGeom& G, const ResArgs& a, int n_chunks, hipStream_t st);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
// Batched phase launch: `kind` selects the projector instantiation (back and
// forward phases); `blocks` is prefix[n_jobs].
hipError_t launch_batch(int phase, int kind, const BatchArgs& b, int blocks, const Tune& t, hipStream_t st);
hipError_t launch_batch_advance(const BatchArgs& b, hipStream_t st);
hipError_t launch_sum_pairs(const double* part, int nblk, double* out, hipStream_t st);
hipError_t launch_resnorm(const float* y, const float* p, int64_t n, double* part, int nblk,
                          hipStream_t st);

}  // namespace ct

// Device-table images of geometries and schedules, for callers that place
// them in device memory of their own (the serving loop's arena): the image's
// size, the image packed into host memory, and the object bound to a copy of
// it in device memory (not freed by the object's destroy).
struct ct_geom;
struct ct_schedule;
size_t geom_table_bytes(const ct_geom* g);
int geom_table_pack(const ct_geom* g, void* dst);
int geom_table_bind(ct_geom* g, void* mem);
size_t sched_table_bytes(const ct_schedule* sc);
int sched_table_pack(const ct_schedule* sc, void* dst);
int sched_table_bind(ct_schedule* sc, void* mem);
// The density count of a geometry whose tables are on the device, enqueued
// on st without waiting; *counts: its device [m][n] table.
int geom_count_async(ct_geom* g, double tau, unsigned long long** counts, hipStream_t st);
