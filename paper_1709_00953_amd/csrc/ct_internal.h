// Internal structures shared by the host runtime (ct_api.cpp) and the gfx950
// kernels (ct_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {

constexpr int kChunk = 256;        // rays per forward work-group
constexpr int kMaxInline = 128;    // row blocks passed by value to a primitive launch
constexpr int kTile2 = 16;         // 2D back-projection tile: 16 x 16 voxels
constexpr int kTile3x = 8, kTile3y = 8, kTile3z = 4;   // 3D tile: 8 x 8 x 4
// Per-view float64 frame: a(3) c(3) e_u(3) e_v(3) n(3) sdd|kappa, 1/sdd, sigma.
constexpr int kViewStride = 24;
enum { kPar2D = 0, kFanFlat = 1, kFanCurved = 2, kCone = 3 };

// One detector tile of a row block: rays (view, v0..v1-1, u0..u1-1).
struct Tile {
    int32_t view, u0, u1, v0, v1;
};

// Up to kChunk consecutive rays of one tile (v-major, u fastest).
struct Chunk {
    int32_t tile;   // global tile index
    int32_t k0;     // first ray within the tile
    int32_t cnt;    // rays in the chunk
    int32_t roff;   // offset of the first ray within its row block
};

// A row block taking part in a launch.  chunk_prefix / slot_prefix are the
// numbers of chunks / rays of the launch that precede this entry.
struct Entry {
    int32_t rb;
    int32_t group;          // group index within the launch (0 for primitives)
    int32_t chunk_prefix;
    int32_t slot_prefix;
};

// Per-(view, bin) constants of a 2D ray, built on the host in float64.
// (dx, dy) is the unit direction used by every 2D kernel.  For the gather
// back-projector, delta = p*B - q*A is the signed distance of the ray from a
// voxel centre whose view-frame coordinates are (A, B), and the clip of the
// ray with the voxel is
//   max(0, min(delta*kx + wx, delta*ky + wy) - max(delta*kx - wx, delta*ky - wy)).
// A zero direction component is marked by wx < 0 (or wy < 0); then kx (ky)
// holds the factor that turns delta into the ray's offset along that axis.
struct Ray2 {
    double p, q, dx, dy;
    float kx, ky, wx, wy;
};

// Device-side geometry, passed by value.
struct DGeom {
    int32_t kind, nx, ny, nz, nu, nv, n_views;
    int32_t dims;
    double vx, vy, vz, ox, oy, oz, pu, pv;
    float radius;                 // voxel half-diagonal (mm)
    const double* view64;         // [n_views][kViewStride]
    const double* bin64;          // [nu][2]  (curved: cos, sin of the bin angle)
    const Ray2* ray2;             // [n_views][nu] (2D kinds)
    const int32_t* view_flags;    // [n_views] bit0: some ray has a zero direction component
    const Tile* tiles;
    const int32_t* rb_tile_ptr;
    const int32_t* tile_roff;     // first ray of the tile within its row block
    const Chunk* chunks;
    const int32_t* rb_chunk_ptr;
};

struct Box {
    int32_t x0, x1, y0, y1, z0, z1;
};

// Forward launch: rays of the entries' row blocks through box J.
struct FwdArgs {
    Box box;
    const Entry* ent;             // device array or nullptr (use inline)
    int32_t n_ent;
    int32_t n_chunks;
    int32_t flags;                // CT_ACCUMULATE
    int32_t mode;                 // 0 single, 1 fused (x,g), 2 count
    const float* x;               // single: full volume
    const float2* xg;             // fused: [group][|J|] (x_J, g_J), J-local
    int32_t vox_J;                // |J|
    float* out;                   // single/fused: ray-indexed (Ax)
    float* q;                     // fused: slot-indexed A g
    double* partial;              // fused: per chunk sum (A g)^2
    unsigned long long* nnz;      // count: [m][n]
    int32_t n_cols, col;          // count: column count and this column
    float tau;                    // count threshold
    Entry inl[kMaxInline];
};

// Back-projection launch: blockIdx.y = group; a group's row blocks are
// entries [gptr[g], gptr[g+1]).
struct BackArgs {
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
    float2* xg;                   // fused: [group][|J|]
    int32_t vox_J;
    double* partial;              // fused: [group][tiles]
    Entry inl[kMaxInline];
};

// Step sizes of one column-block step: group g's ||g||^2 partials are
// pg[g*n_tiles ..], its ||A g||^2 partials the chunks of its entries.
struct StepArgs {
    const Entry* ent;       // step entries (sorted by group)
    const int32_t* gptr;    // group -> entries
    int32_t n_chunks;       // chunks of the step
    int32_t n_tiles;        // back-projection work-groups per group
    const double* pg;       // [G][n_tiles]   ||g||^2 partials
    const double* pq;       // [n_chunks]     ||A g||^2 partials
    const double* beta;     // [G]
    double* mu;             // [G]
};

// Finalize of one column-block step (ray part, then voxel part).
struct FinArgs {
    const Entry* ent;
    int32_t n_ent;
    int32_t n_chunks;
    const double* mu;
    const float* q;
    float* z;               // [n][M]
    float* zJ;              // z + J*M
    const float* y;
    float* r;
    int64_t M;
    int32_t n_cols;
    int32_t refresh;        // 1: r = y - sum_j z^j on the step's rays
    // voxel part
    Box box;
    int32_t vox_J;
    int32_t n_groups;
    const float2* xg;
    float* x;
    int32_t nx, ny;
    Entry inl[1];
};

// Residual refresh over the rays of a list of row blocks.
struct ResArgs {
    const Entry* ent;
    int32_t n_ent;
    const float* z;
    const float* y;
    float* r;
    int64_t M;
    int32_t n_cols;
    Entry inl[1];
};

hipError_t launch_fwd(const DGeom& G, const FwdArgs& a, hipStream_t st);
hipError_t launch_back(const DGeom& G, const BackArgs& a, int n_groups, hipStream_t st);
hipError_t launch_step(const StepArgs& s, int n_groups, hipStream_t st);
hipError_t launch_finalize(const DGeom& G, const FinArgs& f, int vox_blocks, hipStream_t st);
hipError_t launch_residual(const DGeom& G, const ResArgs& a, int n_chunks, hipStream_t st);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_resnorm(const float* y, const float* p, int64_t n, double* part, int nblk,
                          hipStream_t st);

}  // namespace ct
