// gfx950 kernels of the block-iterative CT solver.
//
//  k_fwd      ray-driven Siddon forward projection A_I^J x_J through one
//             column block (Alg. 3 last line; Eq. 12-13).  One lane per ray,
//             consecutive lanes = consecutive detector bins, so the output
//             writes are coalesced along the detector-major ray layout.  The
//             ray is set up in float64 (entry into the box, no division), then
//             walked in float32 box-local coordinates, crossing parameters
//             taken from the plane index rather than by repeated addition.
//             The segment walk forms four segments before their four gathers
//             so that the loads overlap; the 2D fused mode walks slab by slab
//             along the rays' major axis where a chunk allows it (one 16-byte
//             load per slab fetches the two voxels the ray can meet there).
//             The fused mode walks x_J and g_J together (A x and A g in one
//             pass) and emits a float64 partial of ||A g||^2 per work-group;
//             the count mode counts the pairs longer than tau (densities).
//  k_back2/3  gather back-projection (A_I^J)^T r_I (Eq. 7): one lane per
//             voxel, which visits the bins of its shadow in every view of the
//             group and clips each candidate ray against its own box, so no
//             two lanes write the same output and no atomics are needed.
//             The voxel's view-frame offset and each candidate's distance from
//             the voxel centre are formed in float64 (they cancel ~500 mm
//             lever arms); the clip itself is float32.  In 2D a work-group is
//             an 8 x 8 voxel tile whose NW waves take every NW-th view;
//             per (tile, view) one lane derives the frame offsets and a
//             linearised shadow with a rigorous curvature margin, so a voxel's
//             candidate bins cost two FMAs.
//  k_step     mu = beta ||g||^2 / ||A g||^2 (Eq. 11, relaxed) of every group,
//             from the partials in a fixed order.
//  k_finalize z^J_{I_G} = A x + mu A g, residual r = y - sum_j z^j on the
//             touched rays (Sec. II-C), and x_J = mean_G (x_J + mu_G g_G).
//  k_residual r_I = y_I - sum_j z^j_I (epoch-synchronous refresh, reset).
//
// No work-group ever writes an address another one writes (except integer
// atomics of the density count), so every result is reproducible bit for bit.
#include "ct_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>

namespace ct {

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned wave_sum_u(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a 256-lane work-group in a fixed order; result valid in lane 0.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return t;
}

// Load base[i] with a 32-bit unsigned byte offset (lets the compiler use a
// uniform base register plus a per-lane 32-bit offset).  Every array read
// this way lives in global memory; saying so keeps the load a global one even
// when the base pointer was itself read from memory (batched launches).
template <class T>
__device__ __forceinline__ T ldu(const T* base, unsigned i) {
#if defined(__HIP_DEVICE_COMPILE__)
    using GP = const __attribute__((address_space(1))) char*;
    using GT = const __attribute__((address_space(1))) T*;
    return *(GT)((GP)base + i * (unsigned)sizeof(T));
#else
    return base[i];     // host pass: never executed
#endif
}

// Two adjacent (x, g) pairs of a J-local copy, elements i and i + 1: one
// 16-byte load from an 8-byte aligned address (ld_xg2b: at byte offset 8 i).
struct __attribute__((aligned(8))) XG2 {
    float x0, g0, x1, g1;
};
__device__ __forceinline__ XG2 ld_xg2(const float2* base, unsigned i) {
#if defined(__HIP_DEVICE_COMPILE__)
    using GP = const __attribute__((address_space(1))) char*;
    using GT = const __attribute__((address_space(1))) XG2*;
    return *(GT)((GP)base + i * 8u);
#else
    const float2 a = base[i], b = base[i + 1];     // host pass: never executed
    return XG2{a.x, a.y, b.x, b.y};
#endif
}
__device__ __forceinline__ XG2 ld_xg2b(const float2* base, unsigned off) {
#if defined(__HIP_DEVICE_COMPILE__)
    using GP = const __attribute__((address_space(1))) char*;
    using GT = const __attribute__((address_space(1))) XG2*;
    return *(GT)((GP)base + off);
#else
    return ld_xg2(base, off / 8u);                 // host pass: never executed
#endif
}

// Entry i of a launch: inline in the kernel arguments (primitives) or in
// device memory.  The choice is a compile-time property of the argument type
// so that no pointer select makes the compiler copy the arguments to scratch.
// A pointer that is the same in every lane, moved to scalar registers so
// that loads through it can use a scalar base.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

template <class A>
__device__ __forceinline__ Entry get_entry(const A& a, int i) {
    if constexpr (A::kInl) return a.inl[i];
    else return a.ent[i];
}

// Entry that owns launch chunk `bid` (entries sorted by chunk_prefix):
// the last entry whose prefix is <= bid (binary search, uniform per group).
template <class A>
__device__ __forceinline__ int find_entry(const A& a, int bid) {
    int lo = 0, hi = a.n_ent - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (get_entry(a, mid).chunk_prefix <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ const double* view_of(const DGeom& G, int view) {
    return G.view64 + (size_t)view * kViewStride;
}

// Chunk `c` of the launch owned by entry `en` (whole row block, or its window
// on column block `col`).
__device__ __forceinline__ Chunk chunk_of(const DGeom& G, const Entry& en, int c, int windowed, int col) {
    if (windowed) return G.wchunks[G.rbj_chunk_ptr[en.rb * G.n_cols + col] + (c - en.chunk_prefix)];
    return G.chunks[G.rb_chunk_ptr[en.rb] + (c - en.chunk_prefix)];
}

// float64 ray (origin o, unit direction d) of (view, iv, iu).
template <int KIND>
__device__ __forceinline__ void ray_of(const DGeom& G, int view, int iv, int iu, double o[3],
                                       double d[3]) {
    const double* V = view_of(G, view);
    const double u = ((double)iu - 0.5 * (double)(G.nu - 1)) * G.pu;
    if constexpr (KIND == kCone) {
        const double v = ((double)iv - 0.5 * (double)(G.nv - 1)) * G.pv;
        const double sdd = V[15];
        double D0 = fma(v, V[9], fma(u, V[6], sdd * V[12]));
        double D1 = fma(v, V[10], fma(u, V[7], sdd * V[13]));
        double D2 = fma(v, V[11], fma(u, V[8], sdd * V[14]));
        const double inv = 1.0 / sqrt(fma(D0, D0, fma(D1, D1, D2 * D2)));
        d[0] = D0 * inv;
        d[1] = D1 * inv;
        d[2] = D2 * inv;
        o[0] = V[0];
        o[1] = V[1];
        o[2] = V[2];
    } else {
        const Ray2F& R = G.ray2f[(size_t)view * G.nu + iu];
        d[0] = R.dx;
        d[1] = R.dy;
        d[2] = 0.0;
        if constexpr (KIND == kPar2D) {
            o[0] = fma(u, V[6], V[3]);
            o[1] = fma(u, V[7], V[4]);
        } else {
            o[0] = V[0];
            o[1] = V[1];
        }
        o[2] = 0.0;
    }
}

// ----------------------------------------------------------------------------
// K2 / K0: forward projection through box J
// ----------------------------------------------------------------------------
// Forward work-group `bid` of a launch (chunk bid of the entries' rays).
template <int KIND, int MODE, class FA, int KS = kSplit>
__device__ __forceinline__ void fwd_body(const DGeom& G, const FA& a, const int bid) {
    constexpr int DIMS = (KIND == kCone) ? 3 : 2;
    constexpr bool DIVERGENT = (KIND != kPar2D);
    constexpr int U = kWalkU;                  // segments formed before their gathers (padding: xg_pad)
    // the count mode needs whole segment lengths, so it walks each ray in one
    // piece, and in float64: it decides length > tau, and a float32 walk gives
    // a touch of a voxel corner (length 0) lengths of about 1e-7 of the chord
    constexpr int K = (MODE == 2) ? 1 : KS;
    using WT = typename std::conditional<MODE == 2, double, float>::type;
    __shared__ float pacc[K][kChunk], pacc2[K][kChunk];

    const int ei = find_entry(a, bid);
    const Entry en = get_entry(a, ei);
    const int rb = en.rb;
    const Chunk ch = chunk_of(G, en, bid, a.windowed, a.col);
    const int lane = threadIdx.x & (kChunk - 1);
    const int piece = threadIdx.x / kChunk;    // which part of the chord this wave walks
    const bool active = lane < ch.cnt;

    // 2D fused forward: when every ray of the chunk runs at most 45 degrees
    // from one axis and all go the same way along the other, the chunk walks
    // slab by slab along that axis (0: x, 1: y), else (-1) segment by segment
    // (chunks that straddle a diagonal or an axis direction).  Uniform per wave.
    int slab_axis = -1;
    if constexpr (MODE == 1 && DIMS == 2) {
        const int kk = ch.k0 + max(0, min(lane, ch.cnt - 1));
        const Ray2F R = G.ray2f[(size_t)ch.view * G.nu + ch.u0 + kk % ch.w];
        const unsigned long long bx = __ballot(fabs(R.dx) >= fabs(R.dy));
        const int ax = bx == ~0ull ? 0 : (bx == 0ull ? 1 : -1);
        // and every ray of the chunk goes the same way along the other axis
        const unsigned long long bu = __ballot((ax == 0 ? R.dy : R.dx) >= 0.0);
        slab_axis = (bu == ~0ull || bu == 0ull) ? ax : -1;
    }
    // 3D fused forward: the same walk along an xy axis A where every ray of
    // the chunk moves at most one voxel along the other xy axis B and along z
    // per slab of A (at most 45 degrees from A in both planes, in units of
    // the pitches, with a margin), and all go one way along B and one way
    // along z (signs of the direction components after the kernels' zero
    // test, as the walk takes them), in a box whose z slab holds fewer than
    // 2^23 voxels (the walk's index products are 24-bit).
    if constexpr (MODE == 1 && DIMS == 3) {
        const int kk = ch.k0 + max(0, min(lane, ch.cnt - 1));
        const double* V = view_of(G, ch.view);
        const double u = ((double)(ch.u0 + kk % ch.w) - 0.5 * (double)(G.nu - 1)) * G.pu;
        const double v = ((double)(ch.v0 + kk / ch.w) - 0.5 * (double)(G.nv - 1)) * G.pv;
        double D[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            D[c] = fma(v, V[9 + c], fma(u, V[6 + c], V[15] * V[12 + c]));
            if (fabsf((float)(D[c] * V[16])) <= kAxisEpsF) D[c] = 0.0;
        }
        const double m = 1.0 + 1e-6;
        const bool cx = fabs(D[0]) * G.vy >= m * fabs(D[1]) * G.vx && fabs(D[0]) * G.vz >= m * fabs(D[2]) * G.vx;
        const bool cy = fabs(D[1]) * G.vx >= m * fabs(D[0]) * G.vy && fabs(D[1]) * G.vz >= m * fabs(D[2]) * G.vy;
        const unsigned long long bx = __ballot(cx), by = __ballot(cy);
        const int ax = bx == ~0ull ? 0 : (by == ~0ull ? 1 : -1);
        const int nab = (a.box.x1 - a.box.x0) * (a.box.y1 - a.box.y0);
        if (ax >= 0 && nab < (1 << 23)) {
            const unsigned long long bu = __ballot(D[1 - ax] >= 0.0), bz = __ballot(D[2] >= 0.0);
            slab_axis = ((bu == ~0ull || bu == 0ull) && (bz == ~0ull || bz == 0ull)) ? ax : -1;
        }
    }

    float acc = 0.f, acc2 = 0.f;
    unsigned cnt = 0;
    int ray = 0;
    if (active) {
        const int k = ch.k0 + lane;
        const int iv = ch.v0 + k / ch.w;
        const int iu = ch.u0 + k % ch.w;
        const Tile tl{ch.view, 0, 0, 0, 0};
        ray = (tl.view * G.nv + iv) * G.nu + iu;

        // float64 set-up: origin, unit direction, reciprocal direction
        double o[3], d[3], id[3];
        const double* V = view_of(G, tl.view);
        if constexpr (KIND == kCone) {
            const double u = ((double)iu - 0.5 * (double)(G.nu - 1)) * G.pu;
            const double v = ((double)iv - 0.5 * (double)(G.nv - 1)) * G.pv;
            const double sdd = V[15];
            double D[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) D[c] = fma(v, V[9 + c], fma(u, V[6 + c], sdd * V[12 + c]));
            const double inv = 1.0 / sqrt(fma(D[0], D[0], fma(D[1], D[1], D[2] * D[2])));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // the back-projection's test on the same component (D / sdd)
                d[c] = fabsf((float)(D[c] * V[16])) <= kAxisEpsF ? 0.0 : D[c] * inv;
                id[c] = d[c] != 0.0 ? 1.0 / d[c] : 0.0;
                o[c] = V[c];
            }
        } else {
            const Ray2F R = G.ray2f[(size_t)tl.view * G.nu + iu];
            d[0] = R.dx;
            d[1] = R.dy;
            id[0] = R.idx;
            id[1] = R.idy;
            if constexpr (KIND == kPar2D) {
                const double u = ((double)iu - 0.5 * (double)(G.nu - 1)) * G.pu;
                o[0] = fma(u, V[6], V[3]);
                o[1] = fma(u, V[7], V[4]);
            } else {
                o[0] = V[0];
                o[1] = V[1];
            }
        }
        const double h[3] = {G.vx, G.vy, G.vz};
        const double ih[3] = {G.ivx, G.ivy, G.ivz};
        const double org[3] = {G.ox, G.oy, G.oz};
        const int b0[3] = {a.box.x0, a.box.y0, a.box.z0};
        const int b1[3] = {a.box.x1, a.box.y1, a.box.z1};
        double t0 = DIVERGENT ? 0.0 : -INFINITY, t1 = INFINITY;
        bool hit = true;
        double lo[3];
        int zs[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < DIMS; ++c) {
            lo[c] = fma((double)b0[c], h[c], org[c]);
            const double hi = fma((double)b1[c], h[c], org[c]);
            if (d[c] == 0.0) {
                // the ray keeps its origin's coordinate: it lies in one slab,
                // by the half-open rule in float64 (the back-projection takes
                // the same slab)
                const double sl = floor((o[c] - org[c]) * ih[c]);
                const bool in = sl >= (double)b0[c] && sl < (double)b1[c];
                hit = hit && in;
                zs[c] = in ? (int)(sl - (double)b0[c]) : 0;
            } else {
                const double ta = (lo[c] - o[c]) * id[c];
                const double tb = (hi - o[c]) * id[c];
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
        }
        hit = hit && (t1 > t0);
        bool walked = false;
        if constexpr (MODE == 1 && DIMS == 2) {
            if (hit && slab_axis >= 0) {
                // Slab walk.  Along the major axis A the ray crosses one slab
                // of voxels per step; within a slab its coordinate on the
                // other axis B moves by at most one voxel, so it meets at
                // most two voxels there, adjacent along B: one load of the
                // copy whose fast axis is B fetches both.  This wave walks
                // slabs [S0, S1) in traversal order, so the lanes of a wave
                // read one slab row at a time.  Positions are float32 offsets
                // from the plane of slab S0 (tau, mm along the ray) and from
                // the voxel plane jb on B (set up in float64); a slab's length
                // splits at the B plane between its two voxels, clamped to
                // the slab, which also gives a single voxel all of it.
                walked = true;
                const int A = slab_axis, B = 1 - slab_axis;
                const int nx = b1[0] - b0[0], ny = b1[1] - b0[1];
                const int nA = A == 0 ? nx : ny, nB = A == 0 ? ny : nx;
                const int Q = (nA + K - 1) / K;
                const int S0 = __builtin_amdgcn_readfirstlane(piece) * Q, S1 = min(nA, S0 + Q);
                const int nS = S1 - S0;                    // uniform per wave
                if (nS > 0) {
                    const int grp = __builtin_amdgcn_readfirstlane(en.group);
                    const int cs = xg_copy(nx, ny, 1);
                    const float2* xgc = uniform_ptr(a.xg + (size_t)grp * (size_t)a.xg_stride +
                                                    (A == 0 ? (size_t)cs : (size_t)0));
                    const double ia = h[A] * fabs(id[A]);  // mm of ray per slab
                    const double hiA = fma((double)b1[A], h[A], org[A]);
                    const double Cs = ((d[A] > 0.0 ? lo[A] : hiA) - o[A]) * id[A];
                    const double tref = fma((double)S0, ia, Cs);
                    double tlo = fmax(t0 - tref, 0.0);
                    double thi = fmin(t1, fma((double)S1, ia, Cs)) - tref;
                    const bool empty = !(thi > tlo);
                    int jb = 0;
                    double fb64 = 0.5, idb64 = 1e30;
                    float dbf = 0.f;
                    if (empty) {
                        tlo = 0.0;
                        thi = 0.0;
                    } else if (d[B] == 0.0) {
                        jb = zs[B];                        // the ray stays in slab zs of B
                    } else {
                        const double pb = (fma(tref, d[B], o[B]) - lo[B]) * ih[B];
                        const double fl = floor(pb);
                        jb = (int)fl;
                        fb64 = pb - fl;
                        dbf = (float)(d[B] * ih[B]);       // voxels of B per mm of ray
                        idb64 = fmax(fmin(h[B] * id[B], 1e30), -1e30);
                    }
                    const float idb = (float)idb64;
                    // the wave walks the slabs that some lane's ray overlaps: its
                    // lanes' ranges widened by one slab (float rounding), the
                    // union found by a uniform binary search over ballots (lanes
                    // without overlap are neutral)
                    int ulo = nS, uhi = 0;
                    if (!empty) {
                        const double iia = fabs(d[A]) * ih[A];  // slabs per mm of ray
                        ulo = max(0, (int)floor(tlo * iia) - 1);
                        uhi = min(nS, (int)ceil(thi * iia) + 1);
                    }
                    int us = 0, ue = nS;
                    for (int hi = nS; us < hi;) {
                        const int mid = (us + hi) >> 1;
                        if (__ballot(ulo <= mid)) hi = mid;
                        else us = mid + 1;
                    }
                    for (int lo2 = 0; lo2 < ue;) {
                        const int mid = (lo2 + ue) >> 1;
                        if (__ballot(uhi > mid)) lo2 = mid + 1;
                        else ue = mid;
                    }
                    // The B offset is kept as the distance to the next B plane
                    // in the direction of travel, g (float64, then rounded), so
                    // the crossings that lie in the box keep their precision
                    // however small d_B is: going up, voxel lj of a slab ends
                    // at the plane crossed at tau = lj idb + g idb; going down,
                    // voxel lj starts at tau = (lj + 1) idb - g idb.
                    const bool up = d[B] >= 0.0;
                    const double g64 = up ? 1.0 - fb64 : fb64;
                    const float gb = (float)g64;
                    const float nfs = (float)((up ? g64 : -g64) * idb64);
                    const float ias = (float)ia, tl = (float)tlo, th = (float)thi;
                    const int rstep = d[A] > 0.0 ? nB : -nB;
                    // element index of (slab S0 + us, jb); the padding keeps it positive
                    int row = (d[A] > 0.0 ? S0 : nA - 1 - S0) * nB + us * rstep + jb + xg_pad(nx, ny, 1);
                    float uf = (float)us;
                    // voxel (relative to jb) that the ray is in at tau
                    auto vox_at = [&](float t) {
                        return up ? floorf(fmaf(t, dbf, -gb)) + 1.f : floorf(fmaf(t, dbf, gb));
                    };
                    float ts = __builtin_amdgcn_fmed3f(uf * ias, tl, th), fs = vox_at(ts);
                    // DIR 1: every lane's ray goes up B, so the lower voxel of a
                    // slab is the one it starts in; DIR 2: every ray goes down
                    auto walk = [&](auto dir) {
                        constexpr int DIR = decltype(dir)::value;
                        for (int u = us; u < ue; u += U) {
                            int sid[U];
                            float llo[U], lhi[U];
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                // slabs past S1 get zero lengths (tau clamped to th)
                                uf += 1.f;
                                const float te = __builtin_amdgcn_fmed3f(uf * ias, tl, th);
                                const float fe = DIR == 1 ? floorf(fmaf(te, dbf, -gb)) + 1.f
                                                          : floorf(fmaf(te, dbf, gb));
                                const float lj = DIR == 1 ? fs : fe;
                                const float tc = __builtin_amdgcn_fmed3f(
                                    DIR == 1 ? fmaf(lj, idb, nfs) : fmaf(lj + 1.f, idb, nfs), ts, te);
                                const float l1 = tc - ts, l2 = te - tc;
                                llo[q] = DIR == 1 ? l1 : l2;
                                lhi[q] = DIR == 1 ? l2 : l1;
                                sid[q] = row + (int)lj;
                                row += rstep;
                                ts = te;
                                fs = fe;
                            }
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                const XG2 v = ld_xg2(xgc, (unsigned)sid[q]);
                                acc = fmaf(llo[q], v.x0, acc);
                                acc = fmaf(lhi[q], v.x1, acc);
                                acc2 = fmaf(llo[q], v.g0, acc2);
                                acc2 = fmaf(lhi[q], v.g1, acc2);
                            }
                        }
                    };
                    if (__ballot(!up) == 0ull) walk(std::integral_constant<int, 1>{});
                    else walk(std::integral_constant<int, 2>{});
                }
            }
        }
        if constexpr (MODE == 1 && DIMS == 3) {
            if (hit && slab_axis >= 0) {
                // 3D slab walk.  Along the major xy axis A the ray crosses one
                // slab of voxels per step; within a slab it moves by at most
                // one voxel along the other xy axis B and along z, so it meets
                // at most four voxels there, (B, B + 1) x (z, z + 1): two
                // 16-byte loads of the copy whose fast axis is B ([z][A][B])
                // fetch them.  B and z are handled alike, each kept as the
                // float64 distance to its next plane in the direction of
                // travel (then rounded), so crossings keep their precision
                // however small the component; the slab's length splits at the
                // two crossings (each clamped to the slab).
                walked = true;
                const int A = slab_axis, B = 1 - slab_axis;
                const int nx = b1[0] - b0[0], ny = b1[1] - b0[1], nz = b1[2] - b0[2];
                const int nA = A == 0 ? nx : ny, nB = A == 0 ? ny : nx, nAB = nx * ny;
                const int Q = (nA + K - 1) / K;
                const int S0 = __builtin_amdgcn_readfirstlane(piece) * Q, S1 = min(nA, S0 + Q);
                const int nS = S1 - S0;                    // uniform per wave
                if (nS > 0) {
                    const int grp = __builtin_amdgcn_readfirstlane(en.group);
                    const int cs = xg_copy(nx, ny, nz);
                    const float2* xgc = uniform_ptr(a.xg + (size_t)grp * (size_t)a.xg_stride +
                                                    (A == 0 ? (size_t)cs : (size_t)0));
                    const double ia = h[A] * fabs(id[A]);  // mm of ray per slab
                    const double hiA = fma((double)b1[A], h[A], org[A]);
                    const double Cs = ((d[A] > 0.0 ? lo[A] : hiA) - o[A]) * id[A];
                    const double tref = fma((double)S0, ia, Cs);
                    double tlo = fmax(t0 - tref, 0.0);
                    double thi = fmin(t1, fma((double)S1, ia, Cs)) - tref;
                    const bool empty = !(thi > tlo);
                    // minor axes B and z: voxel at tref, its fractional position,
                    // voxels per mm of ray and mm of ray per voxel
                    int jb = 0, jz = 0;
                    double fb64 = 0.5, fz64 = 0.5, idb64 = 1e30, idz64 = 1e30;
                    float dbf = 0.f, dzf = 0.f;
                    if (empty) {
                        tlo = 0.0;
                        thi = 0.0;
                    } else {
                        if (d[B] == 0.0) {
                            jb = zs[B];                    // the ray stays in slab zs of B
                        } else {
                            const double pb = (fma(tref, d[B], o[B]) - lo[B]) * ih[B];
                            const double fl = floor(pb);
                            jb = (int)fl;
                            fb64 = pb - fl;
                            dbf = (float)(d[B] * ih[B]);
                            idb64 = fmax(fmin(h[B] * id[B], 1e30), -1e30);
                        }
                        if (d[2] == 0.0) {
                            jz = zs[2];
                        } else {
                            const double pz = (fma(tref, d[2], o[2]) - lo[2]) * ih[2];
                            const double fl = floor(pz);
                            jz = (int)fl;
                            fz64 = pz - fl;
                            dzf = (float)(d[2] * ih[2]);
                            idz64 = fmax(fmin(h[2] * id[2], 1e30), -1e30);
                        }
                    }
                    // the wave walks the slabs that some lane's ray overlaps
                    // (its lanes' ranges widened by one slab; a uniform binary
                    // search over ballots, lanes without overlap neutral)
                    int ulo = nS, uhi = 0;
                    if (!empty) {
                        const double iia = fabs(d[A]) * ih[A];
                        ulo = max(0, (int)floor(tlo * iia) - 1);
                        uhi = min(nS, (int)ceil(thi * iia) + 1);
                    }
                    int us = 0, ue = nS;
                    for (int hi = nS; us < hi;) {
                        const int mid = (us + hi) >> 1;
                        if (__ballot(ulo <= mid)) hi = mid;
                        else us = mid + 1;
                    }
                    for (int lo2 = 0; lo2 < ue;) {
                        const int mid = (lo2 + ue) >> 1;
                        if (__ballot(uhi > mid)) lo2 = mid + 1;
                        else ue = mid;
                    }
                    const bool up = d[B] >= 0.0, upz = d[2] >= 0.0;
                    const double gb64 = up ? 1.0 - fb64 : fb64, gz64 = upz ? 1.0 - fz64 : fz64;
                    const float gb = (float)gb64, gz = (float)gz64;
                    const float nfs = (float)((up ? gb64 : -gb64) * idb64);
                    const float nzs = (float)((upz ? gz64 : -gz64) * idz64);
                    const float idb = (float)idb64, idz = (float)idz64;
                    // going up, the voxel at tau is floor(tau d + 1 - g) (the +1
                    // folded into the offset); going down, the crossing of the
                    // plane above voxel l is at (l + 1) id - g id, the id folded
                    // into the offset too
                    const float gb1 = up ? 1.f - gb : gb, gz1 = upz ? 1.f - gz : gz;
                    const float nfs1 = up ? nfs : nfs + idb, nzs1 = upz ? nzs : nzs + idz;
                    const float ias = (float)ia, tl = (float)tlo, th = (float)thi;
                    const int rstep = d[A] > 0.0 ? nB : -nB;
                    const unsigned nAB8 = 8u * (unsigned)nAB;
                    // element index of (slab S0 + us, jb, jz); the padding keeps it positive
                    int row = (d[A] > 0.0 ? S0 : nA - 1 - S0) * nB + us * rstep + jb + jz * nAB +
                              xg_pad(nx, ny, nz);
                    float uf = (float)us;
                    float ts = __builtin_amdgcn_fmed3f(uf * ias, tl, th);
                    float fb = floorf(fmaf(ts, dbf, gb1));
                    float fz = floorf(fmaf(ts, dzf, gz1));
                    // DB, DZ 1: every lane's ray goes up B (z), so the lower
                    // voxel of a slab's pair is the one it starts in; 2: down
                    auto walk3 = [&](auto dirb, auto dirz) {
                        constexpr int DB = decltype(dirb)::value, DZ = decltype(dirz)::value;
                        for (int u = us; u < ue; u += U) {
                            int sid[U];
                            float l00[U], l01[U], l10[U], l11[U];   // [B lower, upper][z lower, upper]
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                // slabs past S1 get zero lengths (tau clamped to th)
                                uf += 1.f;
                                const float te = __builtin_amdgcn_fmed3f(uf * ias, tl, th);
                                const float fbe = floorf(fmaf(te, dbf, gb1));
                                const float fze = floorf(fmaf(te, dzf, gz1));
                                const float lb = DB == 1 ? fb : fbe, lz = DZ == 1 ? fz : fze;
                                const float tc = __builtin_amdgcn_fmed3f(fmaf(lb, idb, nfs1), ts, te);
                                const float tz = __builtin_amdgcn_fmed3f(fmaf(lz, idz, nzs1), ts, te);
                                // in the first B voxel on [ts, tc], the second on
                                // [tc, te]; the first z level on [ts, tz], the second
                                // on [tz, te]: the first voxel to min(tc, tz), the last
                                // from max(tc, tz), the one between them (one of the
                                // two mixed ones, the other 0) on [min, max]
                                const float mn = fminf(tc, tz), mx = fmaxf(tc, tz);
                                const float lf[2][2] = {{mn - ts, tc - mn}, {tz - mn, te - mx}};
                                constexpr int bl = DB == 1 ? 0 : 1, zl = DZ == 1 ? 0 : 1;
                                l00[q] = lf[bl][zl];
                                l01[q] = lf[bl][1 - zl];
                                l10[q] = lf[1 - bl][zl];
                                l11[q] = lf[1 - bl][1 - zl];
                                // byte offset (nAB < 2^23, lz small: 24-bit product)
                                sid[q] = (int)((unsigned)(row + (int)lb + __mul24((int)lz, nAB)) << 3);
                                row += rstep;
                                ts = te;
                                fb = fbe;
                                fz = fze;
                            }
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                const XG2 vl = ld_xg2b(xgc, (unsigned)sid[q]);
                                const XG2 vh = ld_xg2b(xgc, (unsigned)sid[q] + nAB8);
                                acc = fmaf(l00[q], vl.x0, acc);
                                acc = fmaf(l10[q], vl.x1, acc);
                                acc = fmaf(l01[q], vh.x0, acc);
                                acc = fmaf(l11[q], vh.x1, acc);
                                acc2 = fmaf(l00[q], vl.g0, acc2);
                                acc2 = fmaf(l10[q], vl.g1, acc2);
                                acc2 = fmaf(l01[q], vh.g0, acc2);
                                acc2 = fmaf(l11[q], vh.g1, acc2);
                            }
                        }
                    };
                    using I1 = std::integral_constant<int, 1>;
                    using I2 = std::integral_constant<int, 2>;
                    const bool bup = __ballot(!up) == 0ull, zup = __ballot(!upz) == 0ull;
                    if (bup) {
                        if (zup) walk3(I1{}, I1{});
                        else walk3(I1{}, I2{});
                    } else {
                        if (zup) walk3(I2{}, I1{});
                        else walk3(I2{}, I2{});
                    }
                }
            }
        }
        if (hit && !walked) {
            // this wave's piece of the chord: [t0 + p L/K, t0 + (p+1) L/K]
            const double Lc = (t1 - t0) / (double)K;
            t0 = fma((double)piece, Lc, t0);
            // box-local walk: ii = voxel, dl = distance (voxel units) to the
            // next plane, inv = mm per voxel along the ray, tk = crossing
            int nb[3], ii[3], sg[3];
            WT dl[3], inv[3], tk[3];
            WT T = (WT)Lc;
#pragma unroll
            for (int c = 0; c < DIMS; ++c) {
                nb[c] = b1[c] - b0[c];
                // the distance to the first plane is formed in float64 before
                // it is rounded: for a ray nearly parallel to the planes of
                // axis c the crossing lies at that distance over a small
                // direction component, so a float32 box-local position
                // (error ~1e-7 voxel) would move it by 1e-7 / |d_c| voxels
                const double ef = (fma(t0, d[c], o[c]) - lo[c]) * ih[c];
                int i = (int)floor(ef);
                if (d[c] < 0.0 && (double)i == ef) i -= 1;
                i = min(max(i, 0), nb[c] - 1);
                ii[c] = d[c] == 0.0 ? zs[c] : i;
                if (d[c] > 0.0) {
                    sg[c] = 1;
                    dl[c] = (WT)((double)(i + 1) - ef);
                    inv[c] = (WT)(h[c] * id[c]);
                    tk[c] = dl[c] * inv[c];
                } else if (d[c] < 0.0) {
                    sg[c] = -1;
                    dl[c] = (WT)(ef - (double)i);
                    inv[c] = (WT)(-h[c] * id[c]);
                    tk[c] = dl[c] * inv[c];
                } else {                       // never crossed: dl * inv stays +inf
                    sg[c] = 0;
                    dl[c] = (WT)1;
                    inv[c] = (WT)INFINITY;
                    tk[c] = (WT)INFINITY;
                }
            }
            // linear voxel index and its step per axis.  The fused path uses
            // the copy whose fast axis is across the view's central ray.
            int step[3];
            int idx;
            const float2* xg = nullptr;
            if constexpr (MODE == 1) {
                const int grp = __builtin_amdgcn_readfirstlane(en.group);
                const double* Vc = view_of(G, tl.view);
                const double cdx = (KIND == kPar2D) ? Vc[0] : Vc[12];
                const double cdy = (KIND == kPar2D) ? Vc[1] : Vc[13];
                const int tr = __builtin_amdgcn_readfirstlane(fabs(cdx) > fabs(cdy) ? 1 : 0);
                const int cs = xg_copy(nb[0], nb[1], DIMS == 3 ? nb[2] : 1);
                xg = uniform_ptr(a.xg + (size_t)grp * (size_t)a.xg_stride + (size_t)tr * (size_t)cs);
                step[0] = tr ? nb[1] : 1;
                step[1] = tr ? 1 : nb[0];
                step[2] = nb[0] * nb[1];
            } else {
                step[0] = 1;
                step[1] = G.nx;
                step[2] = G.nx * G.ny;
            }
            {
                int lin = ii[0] * step[0] + ii[1] * step[1] + (DIMS == 3 ? ii[2] * step[2] : 0);
                if constexpr (MODE == 0)
                    lin += a.box.x0 + a.box.y0 * G.nx + (DIMS == 3 ? a.box.z0 * G.nx * G.ny : 0);
                if constexpr (MODE == 1) lin += xg_pad(nb[0], nb[1], DIMS == 3 ? nb[2] : 1);
                idx = lin;                      // never negative: the padding is in front
            }
            int sst[3];
#pragma unroll
            for (int c = 0; c < DIMS; ++c) sst[c] = sg[c] * step[c];
            const int maxit = (nb[0] + nb[1] + (DIMS == 3 ? nb[2] : 0) + 4 + U - 1) / U;
            WT tau = 0;
            for (int it = 0; it < maxit; ++it) {
                int sid[U];
                WT sl[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    // segment q: from tau to the nearest crossing (or the exit)
                    WT tn = fmin(fmin(tk[0], tk[1]), T);
                    if constexpr (DIMS == 3) tn = fmin(tn, tk[2]);
                    sl[q] = tn - tau;
                    tau = tn;
                    sid[q] = idx;
                    // cross the nearest plane.  Past the exit the lengths are
                    // zero; the fused path then reads the zero padding, the
                    // primitive path is clamped to the box.
                    if constexpr (DIMS == 3) {
                        const bool a0 = tk[0] <= tk[1] && tk[0] <= tk[2];
                        const bool a1 = !a0 && tk[1] <= tk[2];
                        const bool a2 = !a0 && !a1;
                        idx += a0 ? sst[0] : (a1 ? sst[1] : sst[2]);
                        dl[0] = a0 ? dl[0] + 1.f : dl[0];
                        dl[1] = a1 ? dl[1] + 1.f : dl[1];
                        dl[2] = a2 ? dl[2] + 1.f : dl[2];
                        if constexpr (MODE == 0) {
                            ii[0] = a0 ? ii[0] + sg[0] : ii[0];
                            ii[1] = a1 ? ii[1] + sg[1] : ii[1];
                            ii[2] = a2 ? ii[2] + sg[2] : ii[2];
                        }
                    } else {
                        const bool a0 = tk[0] <= tk[1];
                        idx += a0 ? sst[0] : sst[1];
                        dl[0] = a0 ? dl[0] + 1.f : dl[0];
                        dl[1] = a0 ? dl[1] : dl[1] + 1.f;
                        if constexpr (MODE == 0) {
                            ii[0] = a0 ? ii[0] + sg[0] : ii[0];
                            ii[1] = a0 ? ii[1] : ii[1] + sg[1];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < DIMS; ++c) tk[c] = dl[c] * inv[c];
                    if constexpr (MODE == 0) {
                        // keep the caller's array in bounds: stop at the box
                        bool out = false;
#pragma unroll
                        for (int c = 0; c < DIMS; ++c) out = out || (unsigned)ii[c] >= (unsigned)nb[c];
                        if (out) {
                            T = tau;
                            idx = sid[q];
#pragma unroll
                            for (int c = 0; c < DIMS; ++c) ii[c] = min(max(ii[c], 0), nb[c] - 1);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    if constexpr (MODE == 0) {
                        acc = fmaf(sl[q], ldu(a.x, (unsigned)sid[q]), acc);
                    } else if constexpr (MODE == 1) {
                        const float2 v = ldu(xg, (unsigned)sid[q]);
                        acc = fmaf(sl[q], v.x, acc);
                        acc2 = fmaf(sl[q], v.y, acc2);
                    } else {
                        cnt += (sl[q] > a.tau) ? 1u : 0u;
                    }
                }
                if (!(tau < T)) break;
            }
        }
    }

    // the pieces of each ray, added in a fixed order
    if constexpr (K > 1) {
        pacc[piece][lane] = acc;
        if constexpr (MODE == 1) pacc2[piece][lane] = acc2;
        __syncthreads();
        acc = pacc[0][lane];
        if constexpr (MODE == 1) acc2 = pacc2[0][lane];
#pragma unroll
        for (int p = 1; p < K; ++p) {
            acc += pacc[p][lane];
            if constexpr (MODE == 1) acc2 += pacc2[p][lane];
        }
    }
    if constexpr (MODE == 0) {
        if (piece == 0 && active) a.out[ray] = (a.flags & 1) ? a.out[ray] + acc : acc;
    } else if constexpr (MODE == 1) {
        if (piece == 0) {
            if (active) {
                a.out[ray] = acc;
                a.q[en.slot_prefix + ch.roff + lane] = acc2;
            }
            const double t = wave_sum(active ? (double)acc2 * (double)acc2 : 0.0);
            if (lane == 0) a.partial[bid] = t;
        }
    } else {
        const unsigned c = wave_sum_u(cnt);
        if (lane == 0 && c) atomicAdd(a.nnz + (size_t)rb * a.n_cols + a.col, (unsigned long long)c);
    }
}

// Work-group b of n is dispatched to XCD b mod kXcd; give each XCD a
// contiguous run of the launch's chunks (a bijection onto [0, n)), so the
// chunks that one XCD runs together are neighbours in the chunk list.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_run(const int b, const int n) {
    const int q = n / kXcd, r = n % kXcd, x = b % kXcd, i = b / kXcd;
    return x * q + min(x, r) + i;
}

// The 3D fused forward reads a box larger than an XCD's L2; its chunks are
// listed row by row across views, and contiguous runs per XCD let views
// that cross the same voxel planes share them in L2.
template <int KIND, int MODE, int KS = kSplit>
__global__ __launch_bounds__(256) void k_fwd(DGeom G, FwdCore a) {
    const int bid = (KIND == kCone && MODE == 1) ? xcd_run((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    fwd_body<KIND, MODE, FwdCore, KS>(G, a, bid);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_fwd_inl(DGeom G, FwdArgs a) {
    fwd_body<KIND, 0>(G, a, blockIdx.x);
}

// ----------------------------------------------------------------------------
// K1: gather back-projection, 2D
// ----------------------------------------------------------------------------
// Clip length of the ray described by R with the voxel whose centre lies at
// signed distance delta from it: the overlap of its two slab intervals.  The
// difference hs - |delta| is small where the length is on its ramp, and is
// formed in float64 before it is rounded (see Ray2B).
__device__ __forceinline__ float chord2(double delta, const Ray2B& R) {
    return __builtin_amdgcn_fmed3f((float)(R.hs - fabs(delta)) * R.K, 0.f, R.M);   // clamp to [0, M]
}

// Same, for rays with a zero direction component: such a ray lies in one
// slab of that axis (index R.hs) and meets the voxels of that slab only.
__device__ __forceinline__ float chord2_axis(double delta, const Ray2B& R, int ix, int iy) {
    if (R.M < 0.f) {
        const int mine = (R.M == -1.f) ? ix : iy;
        return (double)mine == R.hs ? R.K : 0.f;
    }
    return chord2(delta, R);
}

// Per (tile, view) parameters.  For a voxel at index offset (lx, ly) from the
// tile centre: view-frame offset A = Ac + lx ax + ly ay, B = Bc + lx bx + ly by
// (exact, both are affine in position); bin coordinate of its shadow centre
// ~ bc + lx bxs + ly bys, with W (bins) covering the half-extent of the
// voxel's box (from the gradient), the curvature of the projection over the
// tile and float32 rounding.
struct ViewP {
    double Ac, Bc, ax, ay, bx, by;
    float bc, bxs, bys, W;
    int32_t view, u0, u1, flags;
};

// Curved fan, views with no axis-parallel ray whose candidates stay within
// 2e-2 rad of a reference bin kr near the tile's shadow (flag bit 1): the
// view's frame turned to that bin's ray, stored over (Ac, Bc, ax, ay) of the
// ViewP.  With (p, q) the reference ray's direction terms (its Ray2B), a
// point (A, B) of the view frame lies at lateral offset X = p B - q A and
// depth R = p A + q B from it, both affine in the voxel offsets; the ray of
// bin b, turned from it by e = pu (b - kr) (the bins are equi-angular), passes
// the point at signed distance X cos e - R sin e.  For |e| <= 2e-2 the cubic
// sine and quadratic cosine are exact to 3e-11 and 7e-9 (times distances
// below a metre and a tile), so the distance needs no float64 product per
// candidate, and a candidate reads only K, S, M of its bin and r.
// Where W < 1 a voxel has at most two candidates, b and b + 1 (flag bit 2):
// the second's distance is the first's turned by one pitch,
// X' = X cos pu - Y sin pu with Y = X sin e + R cos e, instead of a second
// polynomial.
struct FanC {
    float Xx, Xy, Yx, Yy;         // X and R per voxel step along x and y
    float Xc, Rc;                 // X and R at the tile centre
    int32_t kr;                   // reference bin
    float pu;                     // bin pitch (rad)
    float cp, sp;                 // cos pu, sin pu
};
static_assert(sizeof(FanC) <= 6 * sizeof(double), "FanC overlays Ac, Bc, ax, ay, bx, by");

template <int KIND>
__device__ __forceinline__ void view_params(const DGeom& G, const Tile& tl, double cx, double cy,
                                            double dt, ViewP& P) {
    const double* V = view_of(G, tl.view);
    const double c0 = 0.5 * (double)(G.nu - 1);
    const double R = (double)G.radius;
    P.view = tl.view;
    P.u0 = tl.u0;
    P.u1 = tl.u1;
    P.flags = G.view_flags[tl.view];
    double bc, bxs, bys, W;
    if constexpr (KIND == kPar2D) {
        // delta(u) = B - u kappa with B = cross(d, p - C): affine, so exact
        P.Ac = 1.0;
        P.ax = P.ay = 0.0;
        P.Bc = V[0] * (cy - V[4]) - V[1] * (cx - V[3]);
        P.bx = -V[1] * G.vx;
        P.by = V[0] * G.vy;
        const double s = 1.0 / (V[15] * G.pu);
        bc = P.Bc * s + c0;
        bxs = P.bx * s;
        bys = P.by * s;
        W = 0.5 * (fabs(bxs) + fabs(bys));          // affine: the box's exact half-extent
    } else {
        const double qx = cx - V[0], qy = cy - V[1];
        P.Ac = fma(qx, V[12], qy * V[13]);
        P.Bc = fma(qx, V[6], qy * V[7]);
        P.ax = V[12] * G.vx;
        P.ay = V[13] * G.vy;
        P.bx = V[6] * G.vx;
        P.by = V[7] * G.vy;
        const double A = P.Ac, B = P.Bc;
        const double rho = sqrt(A * A + B * B);
        const double amin = A - dt;                   // every point of the tile is this deep
        if constexpr (KIND == kFanCurved) {
            // polar angle of the voxel centre; Hessian norm 1/rho^2
            const double rmin = rho - dt;
            const double ir2 = 1.0 / (rho * rho);
            // float32 angle: it only selects candidates (margin 1e-6 rad below)
            bc = (double)atan2f((float)B, (float)A) / G.pu + c0;
            bxs = (A * P.bx - B * P.ax) * ir2 / G.pu;
            bys = (A * P.by - B * P.ay) * ir2 / G.pu;
            // half-extent of a voxel's box from the gradient at the tile centre,
            // plus its variation over the tile, the linearisation of the
            // centre and the voxel's own curvature (Hessian norm <= 1/rmin^2)
            const double hs = 0.5 * (G.vx + G.vy);
            W = (rmin > 1.0001 * R)
                    ? 0.5 * (fabs(bxs) + fabs(bys)) +
                          ((dt * hs + 0.5 * dt * dt + 0.5 * R * R) / ((rmin - R) * (rmin - R)) + 1e-6) / G.pu
                    : 1e9;
        } else {
            // u = sdd * B / A; Hessian norm of B/A <= 2 (1 + |B/A|) / A^2
            const double sdd = V[15];
            const double ia = 1.0 / A;
            bc = sdd * B * ia / G.pu + c0;
            bxs = sdd * (A * P.bx - B * P.ax) * ia * ia / G.pu;
            bys = sdd * (A * P.by - B * P.ay) * ia * ia / G.pu;
            // Hessian bound over the tile's sphere widened by a voxel radius
            const double hs = 0.5 * (G.vx + G.vy);
            const double tbr = (fabs(B) + dt + R) / (amin - R);
            const double H = 2.0 * sdd * (1.0 + tbr) / ((amin - R) * (amin - R)) / G.pu;
            W = (amin > 1.0001 * R)
                    ? 0.5 * (fabs(bxs) + fabs(bys)) + H * (dt * hs + 0.5 * dt * dt + 0.5 * R * R)
                    : 1e9;
        }
    }
    P.bc = (float)bc;
    P.bxs = (float)bxs;
    P.bys = (float)bys;
    P.W = (float)fmin(W, 1e9) + 2e-3f + 1e-6f * fabsf((float)bc);
    if constexpr (KIND == kFanCurved) {
        // candidates lie within W + 4 (|bxs| + |bys|) bins of bc (voxel
        // offsets at most 4 from the tile centre)
        const int kr = min(max((int)floor(bc + 0.5), 0), G.nu - 1);
        const double emax = G.pu * (fabs(bc - kr) + W + 4.0 * (fabs(bxs) + fabs(bys)) + 1.0);
        // and every candidate ray at least 0.02 (in sine) from an axis: K
        // = 1 / |dx dy| then stays below ~50, so the float32 distance's error
        // (< 1e-6 mm) moves a length by at most 5e-5 mm
        const Ray2F& Fr = G.ray2f[(size_t)tl.view * G.nu + kr];
        const bool off_axis = fmin(fabs(Fr.dx), fabs(Fr.dy)) >= emax + 0.02;
        if (!(P.flags & 1) && emax <= 2e-2 && off_axis) {
            const Ray2B& Rr = G.ray2b[(size_t)tl.view * G.nu + kr];
            const double p = Rr.p, q = Rr.q;
            FanC f;
            f.Xx = (float)(p * P.bx - q * P.ax);
            f.Xy = (float)(p * P.by - q * P.ay);
            f.Yx = (float)(p * P.ax + q * P.bx);
            f.Yy = (float)(p * P.ay + q * P.by);
            f.Xc = (float)(p * P.Bc - q * P.Ac);
            f.Rc = (float)(p * P.Ac + q * P.Bc);
            f.kr = kr;
            f.pu = (float)G.pu;
            // pu <= emax <= 2e-2: the series are exact in float32
            const double pu2 = G.pu * G.pu;
            f.cp = (float)fma(pu2, -0.5, 1.0);
            f.sp = (float)(G.pu * fma(pu2, -1.0 / 6.0, 1.0));
            __builtin_memcpy(&P.Ac, &f, sizeof f);
            P.flags |= 2;
            // candidates [ceil(beta - W), floor(beta + W)]: at most two
            // where W < 1 (the margin covers the rounding of beta -+ W)
            if ((float)fmin(W, 1e9) + 2e-3f + 1e-6f * fabsf((float)bc) < 0.999f) P.flags |= 4;
        }
    }
}

// Back-projection work-group for tile `tile` (of n_tiles) of group gi: NW
// waves, each over every NW-th view of the group (NW is a tuning choice).
template <int KIND, class BA, int NW = 4>
__device__ __forceinline__ void back2_body(const DGeom& G, const BA& a, const int gi, const int tile,
                                           const int n_tiles) {
    __shared__ ViewP vp[NW][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int lx = lane & (kTile2 - 1), ly = lane / kTile2;
    const int ix = a.box.x0 + tx * kTile2 + lx, iy = a.box.y0 + ty * kTile2 + ly;
    const bool valid = ix < a.box.x1 && iy < a.box.y1;

    // centre and half-diagonal of the tile's voxels inside the box
    const int xs = a.box.x0 + tx * kTile2, ys = a.box.y0 + ty * kTile2;
    const int nvx = min(kTile2, a.box.x1 - xs), nvy = min(kTile2, a.box.y1 - ys);
    const double tcx = G.ox + ((double)xs + 0.5 * nvx) * G.vx;
    const double tcy = G.oy + ((double)ys + 0.5 * nvy) * G.vy;
    const double hkx = 0.5 * (nvx - 1), hky = 0.5 * (nvy - 1);
    const double dt = sqrt((hkx * G.vx) * (hkx * G.vx) + (hky * G.vy) * (hky * G.vy));
    const float lxf = (float)lx - (float)hkx, lyf = (float)ly - (float)hky;
    const double lxd = (double)lxf, lyd = (double)lyf;

    int e0 = 0, e1 = a.n_ent;
    if (a.gptr) {
        e0 = a.gptr[gi];
        e1 = a.gptr[gi + 1];
    }
    int nt = 0;                                          // views (tiles) of the group
    for (int e = e0; e < e1; ++e) {
        const int rb = get_entry(a, e).rb;
        nt += G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
    }

    float acc = 0.f;
    ViewP* const vpf = &vp[0][0];                        // view slots, flat
    for (int base = 0; base < nt; base += 64 * NW) {
        // Up to four waves a tile, thread i prepares view base + i, so that
        // where the group has fewer views than threads whole waves have none
        // (their lanes would idle through the set-up); wave w then takes
        // views w, w + NW, ...  With eight or sixteen waves, lane l of wave w
        // prepares the view of flat index NW l + w, the set-up of a few views
        // in every wave: one or two waves' 64-lane loads of it measured
        // slower (the paper's 2D setting: 82 against 67 us per launch).  The
        // thread index is formed from the voxel indices (held anyway) and
        // passes through an empty asm statement, so neither it nor the slot's
        // address is held across the loop.
        int slot = (wu << 6) | ((iy - ys) << 3) | (ix - xs);
        asm volatile("" : "+v"(slot));
        const int f = NW >= 8 ? base + NW * (slot & 63) + (slot >> 6) : base + slot;
        if (f < nt) {
            int e = e0, off = f;
            for (;;) {
                const int rb = get_entry(a, e).rb;
                const int cnt = G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
                if (off < cnt) {
                    const Tile tl = G.tiles[G.rb_tile_ptr[rb] + off];
                    view_params<KIND>(G, tl, tcx, tcy, dt, vpf[slot]);
                    break;
                }
                off -= cnt;
                ++e;
            }
        }
        __syncthreads();
        const int nb = min(64, (nt - base - wu + NW - 1) / NW);
        if (valid) {
            for (int j = 0; j < nb; ++j) {
                const ViewP& P = NW >= 8 ? vpf[wu * 64 + j] : vpf[NW * j + wu];
                const int view = __builtin_amdgcn_readfirstlane(P.view);
                const int u0 = __builtin_amdgcn_readfirstlane(P.u0);
                const int u1 = __builtin_amdgcn_readfirstlane(P.u1);
                const int vflags = __builtin_amdgcn_readfirstlane(P.flags);
                const float beta = fmaf(lyf, P.bys, fmaf(lxf, P.bxs, P.bc));
                const int blo = max((int)ceilf(beta - P.W), u0);
                const int bhi = min((int)floorf(beta + P.W), u1 - 1);
                const Ray2B* RB = G.ray2b + (size_t)view * G.nu;
                const float* rr = a.r + (size_t)view * G.nu;
                if (KIND == kFanCurved && (vflags & 4)) {
                    // at most two candidates: bins b0 = blo and b0 + 1, read
                    // where in range and their clips zeroed where not
                    FanC f;
                    __builtin_memcpy(&f, &P.Ac, sizeof f);
                    const float Xs = f.Xc + fmaf(lyf, f.Xy, lxf * f.Xx);
                    const float Rs = f.Rc + fmaf(lyf, f.Yy, lxf * f.Yx);
                    const float4* KS = reinterpret_cast<const float4*>(G.ray2k + (size_t)view * G.nu);
                    const int b0 = min(blo, u1 - 1), b1 = min(b0 + 1, u1 - 1);
                    const float4 k0 = ldu(KS, (unsigned)b0), k1 = ldu(KS, (unsigned)b1);
                    const float r0 = ldu(rr, (unsigned)b0), r1 = ldu(rr, (unsigned)b1);
                    const float e = (float)(b0 - f.kr) * f.pu;
                    const float e2 = e * e;
                    const float sn = e * fmaf(e2, -1.f / 6.f, 1.f);
                    const float cs = fmaf(e2, -0.5f, 1.f);
                    const float d0 = fmaf(cs, Xs, -sn * Rs);
                    const float y0 = fmaf(sn, Xs, cs * Rs);
                    const float d1 = fmaf(d0, f.cp, -y0 * f.sp);
                    const float c0 = __builtin_amdgcn_fmed3f(k0.y - fabsf(d0 * k0.x), 0.f, k0.z);
                    const float c1 = __builtin_amdgcn_fmed3f(k1.y - fabsf(d1 * k1.x), 0.f, k1.z);
                    acc = fmaf(blo <= bhi ? c0 : 0.f, r0, acc);
                    acc = fmaf(blo < bhi ? c1 : 0.f, r1, acc);
                    continue;
                }
                if (KIND == kFanCurved && (vflags & 2)) {
                    if (blo <= bhi) {
                        FanC f;
                        __builtin_memcpy(&f, &P.Ac, sizeof f);
                        const float Xs = f.Xc + fmaf(lyf, f.Xy, lxf * f.Xx);
                        const float Rs = f.Rc + fmaf(lyf, f.Yy, lxf * f.Yx);
                        // K, S, M of bin b
                        const float4* KS = reinterpret_cast<const float4*>(G.ray2k + (size_t)view * G.nu);
                        float ef = (float)(blo - f.kr);      // b - kr, an exact small integer
                        for (int b = blo; b <= bhi; ++b) {
                            const float4 k = ldu(KS, (unsigned)b);
                            const float rv = ldu(rr, (unsigned)b);
                            const float e = ef * f.pu;
                            const float e2 = e * e;
                            const float sn = e * fmaf(e2, -1.f / 6.f, 1.f);
                            const float cs = fmaf(e2, -0.5f, 1.f);
                            const float dlt = fmaf(cs, Xs, -sn * Rs);
                            acc = fmaf(__builtin_amdgcn_fmed3f(k.y - fabsf(dlt * k.x), 0.f, k.z), rv, acc);
                            ef += 1.f;
                        }
                    }
                    continue;
                }
                const double A = fma(lyd, P.ay, fma(lxd, P.ax, P.Ac));
                const double B = fma(lyd, P.by, fma(lxd, P.bx, P.Bc));
                if (vflags & 1) {
                    for (int b = blo; b <= bhi; ++b) {
                        const Ray2B Rb = ldu(RB, (unsigned)b);
                        const double dlt = fma(Rb.p, B, -Rb.q * A);
                        acc = fmaf(chord2_axis(dlt, Rb, ix, iy), ldu(rr, (unsigned)b), acc);
                    }
                } else if (blo <= bhi) {
                    // the next candidate's loads are issued before this one's
                    // clip, so their latency overlaps the arithmetic; the last
                    // candidate reloads its own bin (no branch around the loads)
                    Ray2B Rn = ldu(RB, (unsigned)blo);
                    float rn = ldu(rr, (unsigned)blo);
                    for (int b = blo; b <= bhi; ++b) {
                        const Ray2B Rb = Rn;
                        const float rv = rn;
                        const unsigned bn = (unsigned)min(b + 1, bhi);
                        Rn = ldu(RB, bn);
                        rn = ldu(rr, bn);
                        const double dlt = fma(Rb.p, B, -Rb.q * A);
                        acc = fmaf(chord2(dlt, Rb), rv, acc);
                    }
                }
            }
        }
        __syncthreads();
    }

    // the waves' partial sums, added in a fixed order; the view parameters are
    // dead here and their LDS holds them
    float gsum = acc;
    if constexpr (NW > 1) {
        float* red = reinterpret_cast<float*>(&vp[0][0]);
        red[w * 64 + lane] = acc;
        __syncthreads();
        gsum = red[lane];
#pragma unroll
        for (int k = 1; k < NW; ++k) gsum += red[64 * k + lane];
    }
    const int nxJ = a.box.x1 - a.box.x0;
    if (a.fused) {
        if (w == 0) {
            if (valid) {
                const int nyJ = a.box.y1 - a.box.y0;
                const int lx = ix - a.box.x0, ly = iy - a.box.y0;
                const float2 v = make_float2(a.x[(size_t)iy * G.nx + ix], gsum);
                float2* base = a.xg + (size_t)gi * a.xg_stride + xg_pad(nxJ, nyJ, 1);
                base[ly * nxJ + lx] = v;
                base[xg_copy(nxJ, nyJ, 1) + lx * nyJ + ly] = v;
            }
            const double t = wave_sum(valid ? (double)gsum * (double)gsum : 0.0);
            if (lane == 0) a.partial[(size_t)gi * n_tiles + tile] = t;
        }
    } else if (w == 0 && valid) {
        const size_t gix = (size_t)iy * G.nx + ix;
        a.g[gix] = (a.flags & 1) ? a.g[gix] + gsum : gsum;
    }
}

// At most 64 VGPRs (eight waves per SIMD, the second bound); with four
// waves, 20 KB of LDS: eight work-groups per CU, so a launch of 2048 tiles
// (four groups of a 128 x 256 block) is resident in one round.  Eight or
// sixteen waves per tile (up to 80 KB of LDS) spread a small launch's views
// over more SIMDs.  One wave per tile, and the standalone products (entries
// inline in the arguments), keep a lane's curved-fan state in registers at
// seven waves per SIMD (72 VGPRs).
constexpr int back2_waves(int nw, bool inl) { return (nw == 1 || (inl && nw <= 4)) ? 7 : (nw <= 4 ? 8 : 32 / nw); }
template <int KIND, class BA, int NW>
__global__ __launch_bounds__(64 * NW, back2_waves(NW, BA::kInl)) void k_back2(DGeom G, BA a) {
    back2_body<KIND, BA, NW>(G, a, blockIdx.y, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------
// K1: gather back-projection, 3D cone
// ----------------------------------------------------------------------------
// View frame of a cone view: source S, unit detector normal n, detector axes
// e_u, e_v (orthonormal), source-detector distance sdd.  A voxel centre c has
// frame coordinates A = (c-S).n, Bu = (c-S).e_u, Bv = (c-S).e_v.  The ray of
// bin (u, v) is S + t D~ with D~ = n + (u/sdd) e_u + (v/sdd) e_v; at depth
// A + s it lies at  s D~ - du e_u - dv e_v  from c, where du = Bu - A u/sdd and
// dv = Bv - A v/sdd.  Its x/y/z slabs of the voxel are s-intervals centred on
//   s_k = du a_k + dv b_k,  a_k = e_u,k / D~_k,  b_k = e_v,k / D~_k
// with half-widths w_k = h_k / |D~_k|, and the clip length is
//   |D~| max(0, min_k(s_k + w_k) - max_k(s_k - w_k)).
// A work-group owns an 8 x 8 x 4 voxel tile (one voxel per lane) and walks the
// views of the group.  Per (tile, view), one lane forms in float64 the tile
// centre's frame coordinates and the bases of du and dv along the detector.
// Each voxel's candidate window is its shadow centre sdd B / A plus the
// half-extent of its box from the gradient at its centre, widened by the
// remainder (Hessian of B/A, norm <= 2 (1 + |B/A|) / A^2, over the tile's
// bounding sphere, times R^2 / 2); du at the window's first bin needs one
// float64 FMA (it cancels lever arms of the source distance), the steps along
// the window are float32.  The
// per-ray constants of the tile's detector window (the bounding rectangle of
// its box's projected corners) and r are staged in LDS, and each voxel runs
// one flattened loop over its window.
struct ViewP3 {
    double D0u, D0v, slu, slv;    // du = D0u + (iu - uref) slu + dBu - dA us(iu) (same for v)
    float ax, ay, az;             // A, Bu, Bv per voxel step in x, y, z
    float bux, buy, buz, bvx, bvy, bvz;
    float At, But, Bvt;           // tile centre (float32: shadow windows only)
    float su, sv;                 // sdd / pu, sdd / pv
    float e2u, e2v;               // curvature remainder over a voxel + float32 margins (bins)
    float usr, vsr, dus, dvs;     // u/sdd at uref and per bin (same for v)
    float eu[3], ev[3], n[3];
    int32_t view, fu0, fu1, fv0, fv1;     // detector window [fu0, fu1) x [fv0, fv1)
    int32_t uref, vref, flags;
    int32_t sk[3];                // the source's slab per axis (rays with a zero component stay in it)
    int32_t chh;                  // window rows per staging pass
};

constexpr int kRayC = 256;        // staged rays per pass

__device__ __forceinline__ void view_params3(const DGeom& G, const Tile& tl, const double tc[3],
                                             const double tr, const double tlo[3], const double thi[3],
                                             ViewP3& P) {
    const double* V = view_of(G, tl.view);
    const double sdd = V[15], isdd = V[16];
    const double q[3] = {tc[0] - V[0], tc[1] - V[1], tc[2] - V[2]};
    const double At = fma(q[0], V[12], fma(q[1], V[13], q[2] * V[14]));
    const double But = fma(q[0], V[6], fma(q[1], V[7], q[2] * V[8]));
    const double Bvt = fma(q[0], V[9], fma(q[1], V[10], q[2] * V[11]));
    const double h[3] = {G.vx, G.vy, G.vz};
    P.ax = (float)(V[12] * h[0]);
    P.ay = (float)(V[13] * h[1]);
    P.az = (float)(V[14] * h[2]);
    P.bux = (float)(V[6] * h[0]);
    P.buy = (float)(V[7] * h[1]);
    P.buz = (float)(V[8] * h[2]);
    P.bvx = (float)(V[9] * h[0]);
    P.bvy = (float)(V[10] * h[1]);
    P.bvz = (float)(V[11] * h[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.eu[k] = (float)V[6 + k];
        P.ev[k] = (float)V[9 + k];
        P.n[k] = (float)V[12 + k];
    }
    P.view = tl.view;
    P.flags = G.view_flags[tl.view];
    {
        const double org[3] = {G.ox, G.oy, G.oz}, ih[3] = {G.ivx, G.ivy, G.ivz};
#pragma unroll
        for (int k = 0; k < 3; ++k) P.sk[k] = (int)fmin(fmax(floor((V[k] - org[k]) * ih[k]), -1e9), 1e9);
    }
    P.At = (float)At;
    P.But = (float)But;
    P.Bvt = (float)Bvt;
    P.su = (float)(sdd / G.pu);
    P.sv = (float)(sdd / G.pv);
    const double c0u = 0.5 * (double)(G.nu - 1), c0v = 0.5 * (double)(G.nv - 1);
    const double R = (double)G.radius;
    int u0 = tl.u0, u1 = tl.u1, v0 = tl.v0, v1 = tl.v1;
    double bu = c0u, bv = c0v, e2u = 1e9, e2v = 1e9;
    if (At > 1.0001 * (tr + R)) {
        const double tu = But / At, tv = Bvt / At;
        bu = sdd * tu / G.pu + c0u;
        bv = sdd * tv / G.pv + c0v;
        // detector window of the tile: its box lies in front of the source, so
        // the box's image is the convex hull of its eight projected corners
        double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
        const double hx = 0.5 * (thi[0] - tlo[0]), hy = 0.5 * (thi[1] - tlo[1]), hz = 0.5 * (thi[2] - tlo[2]);
#pragma unroll 1
        for (int c = 0; c < 8; ++c) {
            const double sx = (c & 1) ? hx : -hx, sy = (c & 2) ? hy : -hy, sz = (c & 4) ? hz : -hz;
            const double ia = 1.0 / fma(sz, V[14], fma(sy, V[13], fma(sx, V[12], At)));
            const double cu = sdd * fma(sz, V[8], fma(sy, V[7], fma(sx, V[6], But))) * ia;
            const double cv = sdd * fma(sz, V[11], fma(sy, V[10], fma(sx, V[9], Bvt))) * ia;
            umin = fmin(umin, cu);
            umax = fmax(umax, cu);
            vmin = fmin(vmin, cv);
            vmax = fmax(vmax, cv);
        }
        u0 = max(u0, (int)fmax(ceil(umin / G.pu + c0u - 1e-3), -1.0));
        u1 = min(u1, (int)fmin(floor(umax / G.pu + c0u + 1e-3), 2e9) + 1);
        v0 = max(v0, (int)fmax(ceil(vmin / G.pv + c0v - 1e-3), -1.0));
        v1 = min(v1, (int)fmin(floor(vmax / G.pv + c0v + 1e-3), 2e9) + 1);
        // second-order remainder of a voxel's shadow about its own centre:
        // Hessian norm of sdd B / A over the tile's sphere times R^2 / 2
        const double amin = At - tr - R;
        const double Hu = 2.0 * sdd * (1.0 + (fabs(But) + tr + R) / amin) / (amin * amin) / G.pu;
        const double Hv = 2.0 * sdd * (1.0 + (fabs(Bvt) + tr + R) / amin) / (amin * amin) / G.pv;
        e2u = 0.5 * Hu * R * R;
        e2v = 0.5 * Hv * R * R;
    }
    P.fu0 = u0;
    P.fu1 = max(u0, u1);
    P.fv0 = v0;
    P.fv1 = max(v0, v1);
    P.chh = max(1, kRayC / max(1, min(P.fu1 - P.fu0, kRayC)));
    // rays of the window with a direction component below kNearAxis (D~
    // units, |D~| >= 1) take the float64 candidate path: the component is
    // affine in (u, v), so its smallest magnitude over the window is at a
    // corner unless it changes sign there
    if (P.fu1 > P.fu0 && P.fv1 > P.fv0) {
        const double ua = ((double)P.fu0 - c0u) * G.pu, ub = ((double)(P.fu1 - 1) - c0u) * G.pu;
        const double va = ((double)P.fv0 - c0v) * G.pv, vb = ((double)(P.fv1 - 1) - c0v) * G.pv;
        int nm = 0;                                  // the axes that have such rays
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double c = V[12 + k], eu = V[6 + k] * isdd, ev = V[9 + k] * isdd;
            const double d00 = fma(va, ev, fma(ua, eu, c)), d01 = fma(vb, ev, fma(ua, eu, c));
            const double d10 = fma(va, ev, fma(ub, eu, c)), d11 = fma(vb, ev, fma(ub, eu, c));
            const double lo = fmin(fmin(d00, d01), fmin(d10, d11));
            const double hi = fmax(fmax(d00, d01), fmax(d10, d11));
            if (lo < kNearAxis && hi > -kNearAxis) nm |= 1 << k;
        }
        if (nm) P.flags |= 4 | (nm << 8);
    }
    // plus the float32 rounding of the voxel's shadow centre and half-extent
    // (|beta| <= a few thousand bins)
    P.e2u = (float)fmin(e2u, 1e9) + 2e-3f + 2e-6f * fabsf((float)bu);
    P.e2v = (float)fmin(e2v, 1e9) + 2e-3f + 2e-6f * fabsf((float)bv);
    // bases of du, dv: reference bins near the tile centre's shadow
    const int uref = (int)fmin(fmax(rint(bu), -1e6), 1e6), vref = (int)fmin(fmax(rint(bv), -1e6), 1e6);
    const double usr = ((double)uref - c0u) * G.pu * isdd, vsr = ((double)vref - c0v) * G.pv * isdd;
    P.uref = uref;
    P.vref = vref;
    P.D0u = fma(-At, usr, But);
    P.D0v = fma(-At, vsr, Bvt);
    P.slu = -At * G.pu * isdd;
    P.slv = -At * G.pv * isdd;
    P.usr = (float)usr;
    P.vsr = (float)vsr;
    P.dus = (float)(G.pu * isdd);
    P.dvs = (float)(G.pv * isdd);
}

// Clipped parameter extent of a staged ray in the voxel at offsets (du, dv)
// (times the ray's |d| it is the intersection length).  Views whose rays have
// a zero or small direction component take clip3_precise instead.
__device__ __forceinline__ float clip3(float du, float dv, const float4& q0, const float4& q1,
                                       const float4& q2) {
    const float s0 = fmaf(du, q0.x, dv * q1.x);
    const float s1 = fmaf(du, q0.y, dv * q1.y);
    const float s2 = fmaf(du, q0.z, dv * q1.z);
    const float lo = fmaxf(fmaxf(s0 - q0.w, s1 - q1.w), s2 - q2.x);
    const float hi = fminf(fminf(s0 + q0.w, s1 + q1.w), s2 + q2.x);
    return fmaxf(hi - lo, 0.f);
}

// The same extent with the slab bounds' numerators in float64.  For a ray
// whose component D~_k is small the bound (du e_u,k + dv e_v,k -+ h_k) / D~_k
// of axis k moves by the numerator's error over |D~_k|, and float32 offsets
// (error ~1e-7 mm) would move it by up to 1e-7 / |D~_k| mm; here du, dv and the
// numerators are float64 and only the quotient is float32 (relative error).
// A zero component (the kernels' rule: |D~_k| rounded to float32 <= kAxisEpsF)
// keeps the ray in the source's slab sk of that axis.  (Au, Bu, Bv): the
// voxel centre's view-frame coordinates in float64.
__device__ __forceinline__ float clip3_precise(const double* V, double u, double v, double Av,
                                               double Bu, double Bv, const double h[3],
                                               const int vi[3], const int sk[3]) {
    const double isdd = V[16];
    const double du = fma(-Av, u * isdd, Bu), dv = fma(-Av, v * isdd, Bv);
    float lo = -INFINITY, hi = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double Dk = fma(v, V[9 + k], fma(u, V[6 + k], V[15] * V[12 + k]));
        const float dk = (float)(Dk * isdd);
        if (fabsf(dk) <= kAxisEpsF) {
            if (vi[k] != sk[k]) hi = -INFINITY;
        } else {
            const double num = fma(du, V[6 + k], dv * V[9 + k]);
            const float ik = __builtin_amdgcn_rcpf(dk);
            const float a = (float)(num - h[k]) * ik, b = (float)(num + h[k]) * ik;
            lo = fmaxf(lo, fminf(a, b));
            hi = fminf(hi, fmaxf(a, b));
        }
    }
    return fmaxf(hi - lo, 0.f);
}

// The same with only the axes of mask nm (those whose window holds a ray
// with a small or zero component) in float64; the other axes' rays all have
// components of at least kNearAxis, so their bounds take the staged float32
// form (q0, q1, q2 as in clip3) on du, dv rounded from float64.
__device__ __forceinline__ float clip3_mixed(const double* V, double u, double v, double Av, double Bu,
                                             double Bv, const double h[3], const int vi[3], const int sk[3],
                                             int nm, const float4& q0, const float4& q1, const float4& q2) {
    const double isdd = V[16];
    const double du = fma(-Av, u * isdd, Bu), dv = fma(-Av, v * isdd, Bv);
    const float duf = (float)du, dvf = (float)dv;
    const float al[3] = {q0.x, q0.y, q0.z}, be[3] = {q1.x, q1.y, q1.z}, w[3] = {q0.w, q1.w, q2.x};
    float lo = -INFINITY, hi = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (nm & (1 << k)) {
            const double Dk = fma(v, V[9 + k], fma(u, V[6 + k], V[15] * V[12 + k]));
            const float dk = (float)(Dk * isdd);
            if (fabsf(dk) <= kAxisEpsF) {
                if (vi[k] != sk[k]) hi = -INFINITY;
            } else {
                const double num = fma(du, V[6 + k], dv * V[9 + k]);
                const float ik = __builtin_amdgcn_rcpf(dk);
                const float a = (float)(num - h[k]) * ik, b = (float)(num + h[k]) * ik;
                lo = fmaxf(lo, fminf(a, b));
                hi = fminf(hi, fmaxf(a, b));
            }
        } else {
            const float sk2 = fmaf(duf, al[k], dvf * be[k]);
            lo = fmaxf(lo, sk2 - w[k]);
            hi = fminf(hi, sk2 + w[k]);
        }
    }
    return fmaxf(hi - lo, 0.f);
}

// float4 at byte offset `b` of an LDS array
__device__ __forceinline__ float4 lds_f4(const float4* base, int b) {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(base) + b);
}

template <class BA>
__device__ __forceinline__ void back3_body(const DGeom& G, const BA& a, const int gi, const int bt,
                                           const int n_tiles) {
    __shared__ ViewP3 vp[64];
    __shared__ float4 rc0[kRayC], rc1[kRayC], rc2[kRayC];
    __shared__ double sh[4];
    const int t = threadIdx.x;
    const int tx = bt % a.tiles_x;
    const int ty = (bt / a.tiles_x) % a.tiles_y;
    const int tz = bt / (a.tiles_x * a.tiles_y);
    const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const int ix = a.box.x0 + tx * kTile3x + lx;
    const int iy = a.box.y0 + ty * kTile3y + ly;
    const int iz = a.box.z0 + tz * kTile3z + lz;
    const bool valid = ix < a.box.x1 && iy < a.box.y1 && iz < a.box.z1;
    const int vi[3] = {ix, iy, iz};

    // tile centre, bounding-sphere radius, and this voxel's offset from the centre
    const int xs = a.box.x0 + tx * kTile3x, ys = a.box.y0 + ty * kTile3y, zs = a.box.z0 + tz * kTile3z;
    const int nvx = min(kTile3x, a.box.x1 - xs), nvy = min(kTile3y, a.box.y1 - ys);
    const int nvz = min(kTile3z, a.box.z1 - zs);
    const double tc[3] = {G.ox + ((double)xs + 0.5 * nvx) * G.vx, G.oy + ((double)ys + 0.5 * nvy) * G.vy,
                          G.oz + ((double)zs + 0.5 * nvz) * G.vz};
    const double trad = 0.5 * sqrt((nvx * G.vx) * (nvx * G.vx) + (nvy * G.vy) * (nvy * G.vy) +
                                   (nvz * G.vz) * (nvz * G.vz)) * (1.0 + 1e-9);
    const double tlo[3] = {G.ox + (double)xs * G.vx, G.oy + (double)ys * G.vy, G.oz + (double)zs * G.vz};
    const double thi[3] = {G.ox + (double)(xs + nvx) * G.vx, G.oy + (double)(ys + nvy) * G.vy,
                           G.oz + (double)(zs + nvz) * G.vz};
    const float ox = (float)lx - 0.5f * (float)(nvx - 1), oy = (float)ly - 0.5f * (float)(nvy - 1);
    const float oz = (float)lz - 0.5f * (float)(nvz - 1);
    const float hh[3] = {(float)(0.5 * G.vx), (float)(0.5 * G.vy), (float)(0.5 * G.vz)};
    const double pu = G.pu, pv = G.pv;
    const double c0u = 0.5 * (double)(G.nu - 1), c0v = 0.5 * (double)(G.nv - 1);

    int e0 = 0, e1 = a.n_ent;
    if (a.gptr) {
        e0 = a.gptr[gi];
        e1 = a.gptr[gi + 1];
    }
    int nt = 0;                                          // views (tiles) of the group
    for (int e = e0; e < e1; ++e) {
        const int rb = get_entry(a, e).rb;
        nt += G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
    }

    float acc = 0.f;
    for (int base = 0; base < nt; base += 64) {
        if (t < 64 && base + t < nt) {
            int e = e0, off = base + t;
            for (;;) {
                const int rb = get_entry(a, e).rb;
                const int cnt = G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
                if (off < cnt) {
                    view_params3(G, G.tiles[G.rb_tile_ptr[rb] + off], tc, trad, tlo, thi, vp[t]);
                    break;
                }
                off -= cnt;
                ++e;
            }
        }
        __syncthreads();
        const int nb = min(64, nt - base);
        for (int j = 0; j < nb; ++j) {
            const ViewP3& P = vp[j];
            const int view = __builtin_amdgcn_readfirstlane(P.view);
            const int fu0 = __builtin_amdgcn_readfirstlane(P.fu0), fu1 = __builtin_amdgcn_readfirstlane(P.fu1);
            const int fv0 = __builtin_amdgcn_readfirstlane(P.fv0), fv1 = __builtin_amdgcn_readfirstlane(P.fv1);
            // zero or small direction components in the window (flag bits 0, 2)
            const bool near = (__builtin_amdgcn_readfirstlane(P.flags) & 5) != 0;
            const int fw = fu1 - fu0, fh = fv1 - fv0;
            if (fw <= 0 || fh <= 0) continue;
            const float* rview = uniform_ptr(a.r + (size_t)view * G.nv * G.nu);
            // this voxel's offsets and candidate window: its shadow centre
            // sdd B / A and the half-extent of its box, from the gradient at
            // its own centre, plus the remainder e2
            const float dA = fmaf(oz, P.az, fmaf(oy, P.ay, ox * P.ax));
            const float dBu = fmaf(oz, P.buz, fmaf(oy, P.buy, ox * P.bux));
            const float dBv = fmaf(oz, P.bvz, fmaf(oy, P.bvy, ox * P.bvx));
            const float iA = __builtin_amdgcn_rcpf(P.At + dA);
            const float tu = (P.But + dBu) * iA, tv = (P.Bvt + dBv) * iA;
            float hu = 0.f, hv = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                hu = fmaf(hh[k], fabsf(fmaf(-tu, P.n[k], P.eu[k])), hu);
                hv = fmaf(hh[k], fabsf(fmaf(-tv, P.n[k], P.ev[k])), hv);
            }
            const float betu = fmaf(P.su, tu, (float)c0u), betv = fmaf(P.sv, tv, (float)c0v);
            const float Wu = fmaf(P.su * iA, hu, P.e2u), Wv = fmaf(P.sv * iA, hv, P.e2v);
            const int ulo = valid ? (int)ceilf(betu - Wu) : 1, uhi = valid ? (int)floorf(betu + Wu) : 0;
            const int vlo = valid ? (int)ceilf(betv - Wv) : 1, vhi = valid ? (int)floorf(betv + Wv) : 0;
            const float stu = fmaf(-dA, P.dus, (float)P.slu), stv = fmaf(-dA, P.dvs, (float)P.slv);
            // the detector window in passes of at most kRayC rays
            const int cw = min(fw, kRayC), chh = __builtin_amdgcn_readfirstlane(P.chh);
            for (int cv0 = fv0; cv0 < fv1; cv0 += chh) {
                const int cv1 = min(fv1, cv0 + chh);
                for (int cu0 = fu0; cu0 < fu1; cu0 += cw) {
                    const int cu1 = min(fu1, cu0 + cw);
                    const int pw = cu1 - cu0, np = pw * (cv1 - cv0);
                    // row of lane t in the pass: (t + 1/2) / pw lies at least 1/(2 pw)
                    // from an integer, far beyond the rounding of rcp and the
                    // product (a few 1e-7 relative) for t < 256
                    const float ipw = __builtin_amdgcn_rcpf((float)pw);
                    __syncthreads();                    // previous pass fully read
                    if (t < np) {
                        const int row = (int)(((float)t + 0.5f) * ipw);
                        const int iu = cu0 + (t - row * pw), iv = cv0 + row;
                        const double u = ((double)iu - c0u) * pu, v = ((double)iv - c0v) * pv;
                        const double* V = view_of(G, view);
                        float d[3];
                        int zero = 0;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            const double Dk = fma(v, V[9 + k], fma(u, V[6 + k], V[15] * V[12 + k]));
                            d[k] = (float)(Dk * V[16]);
                            zero |= (fabsf(d[k]) <= kAxisEpsF) ? (1 << k) : 0;
                        }
                        float al[3], be[3], w[3];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            const float inv = (zero >> k) & 1 ? 0.f : __builtin_amdgcn_rcpf(d[k]);
                            al[k] = P.eu[k] * inv;
                            be[k] = P.ev[k] * inv;
                            w[k] = (zero >> k) & 1 ? INFINITY : hh[k] * fabsf(inv);
                        }
                        const float nrm = __builtin_amdgcn_sqrtf(fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2])));
                        const float rv = ldu(rview, (unsigned)(iv * G.nu + iu));
                        rc0[t] = make_float4(al[0], al[1], al[2], w[0]);
                        rc1[t] = make_float4(be[0], be[1], be[2], w[1]);
                        // |d| r: the length scale and the residual in one factor
                        rc2[t] = make_float4(w[2], nrm * rv, 0.f, __int_as_float(zero));
                    }
                    __syncthreads();
                    const int ua = max(ulo, cu0), ub = min(uhi, cu1 - 1);
                    const int va = max(vlo, cv0), vb = min(vhi, cv1 - 1);
                    const int nu_w = ub - ua + 1, n_c = (ua <= ub && va <= vb) ? nu_w * (vb - va + 1) : 0;
                    if (n_c == 0) continue;
                    // du, dv at (ua, va): float64 base of the tile plus the
                    // voxel's small float32 offsets
                    const float du0 = (float)fma((double)(ua - P.uref), P.slu, P.D0u) +
                                      fmaf(-dA, fmaf((float)(ua - P.uref), P.dus, P.usr), dBu);
                    const float dv0 = (float)fma((double)(va - P.vref), P.slv, P.D0v) +
                                      fmaf(-dA, fmaf((float)(va - P.vref), P.dvs, P.vsr), dBv);
                    // the rectangle row by row in one flat loop: the column
                    // offset (an exact small integer) is kept as a float, dv
                    // steps by stv at the end of a row, and the LDS byte
                    // offset jumps to the next row there (views with small
                    // direction components: the float64 path, a uniform branch)
                    const int lb0 = ((va - cv0) * pw + (ua - cu0)) * 16;
                    const int lb_end = lb0 + (vb - va + 1) * pw * 16;   // where the last wrap lands
                    const int jump = (pw - nu_w + 1) * 16;
                    const float last = (float)(nu_w - 1);
                    if (near) {
                        // float64 numerators (clip3_precise): the voxel centre's
                        // view-frame coordinates from the tile centre's (recovered
                        // from the float64 bases) plus its offsets
                        const double* V = view_of(G, view);
                        const double At = -P.slu * V[15] / pu;
                        const double Bu = fma(At, ((double)P.uref - c0u) * pu * V[16], P.D0u) +
                                          fma((double)oz * G.vz, V[8], fma((double)oy * G.vy, V[7], (double)ox * G.vx * V[6]));
                        const double Bv = fma(At, ((double)P.vref - c0v) * pv * V[16], P.D0v) +
                                          fma((double)oz * G.vz, V[11], fma((double)oy * G.vy, V[10], (double)ox * G.vx * V[9]));
                        const double Av = At + fma((double)oz * G.vz, V[14], fma((double)oy * G.vy, V[13], (double)ox * G.vx * V[12]));
                        const double h64[3] = {0.5 * G.vx, 0.5 * G.vy, 0.5 * G.vz};
                        const int nm = (__builtin_amdgcn_readfirstlane(P.flags) >> 8) & 7;
                        for (int iv = va; iv <= vb; ++iv) {
                            const double v = ((double)iv - c0v) * pv;
                            for (int iu = ua; iu <= ub; ++iu) {
                                const int lbc = ((iv - cv0) * pw + (iu - cu0)) * 16;
                                const float4 q2 = lds_f4(rc2, lbc);
                                const double u = ((double)iu - c0u) * pu;
                                if (nm == 7) {
                                    acc = fmaf(clip3_precise(V, u, v, Av, Bu, Bv, h64, vi, P.sk), q2.y, acc);
                                } else {
                                    const float4 q0 = lds_f4(rc0, lbc), q1 = lds_f4(rc1, lbc);
                                    acc = fmaf(clip3_mixed(V, u, v, Av, Bu, Bv, h64, vi, P.sk, nm, q0, q1, q2),
                                               q2.y, acc);
                                }
                            }
                        }
                    } else {
                        float kuf = 0.f, dv = dv0;
                        int lb = lb0;
                        do {
                            const float du = fmaf(kuf, stu, du0);
                            const float4 q0 = lds_f4(rc0, lb), q1 = lds_f4(rc1, lb), q2 = lds_f4(rc2, lb);
                            acc = fmaf(clip3(du, dv, q0, q1, q2), q2.y, acc);
                            const bool wrap = kuf == last;
                            kuf = wrap ? 0.f : kuf + 1.f;
                            dv = wrap ? dv + stv : dv;
                            lb += wrap ? jump : 16;
                        } while (lb != lb_end);
                    }
                }
            }
        }
        __syncthreads();
    }

    const int nxJ = a.box.x1 - a.box.x0, nyJ = a.box.y1 - a.box.y0;
    const size_t gix = ((size_t)iz * G.ny + iy) * G.nx + ix;
    if (a.fused) {
        if (valid) {
            const int nzJ = a.box.z1 - a.box.z0;
            const int jx = ix - a.box.x0, jy = iy - a.box.y0, jz = iz - a.box.z0;
            const float2 v = make_float2(a.x[gix], acc);
            float2* basep = a.xg + (size_t)gi * a.xg_stride + xg_pad(nxJ, nyJ, nzJ);
            basep[(jz * nyJ + jy) * nxJ + jx] = v;
            basep[xg_copy(nxJ, nyJ, nzJ) + (jz * nxJ + jx) * nyJ + jy] = v;
        }
        const double p = valid ? (double)acc * (double)acc : 0.0;
        const double tsum = block_sum256(p, sh);
        if (threadIdx.x == 0) a.partial[(size_t)gi * n_tiles + bt] = tsum;
    } else if (valid) {
        a.g[gix] = (a.flags & 1) ? a.g[gix] + acc : acc;
    }
}

// Six work-groups per CU (the LDS limit; at most 80 VGPRs, six waves per
// SIMD): the kernel waits on its staging loads and barriers, and two more
// resident work-groups than at 128 VGPRs hide them (the register spills this
// costs are in the once-per-64-views parameter set-up only)
template <class BA>
__global__ __launch_bounds__(256, 6) void k_back3(DGeom G, BA a) {
    back3_body(G, a, blockIdx.y, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------
// K1: gather back-projection, cone views with detector columns along z
// ----------------------------------------------------------------------------
// When e_v = +-z and e_u, n lie in the xy plane (a circular orbit about the z
// axis), every ray of detector column u lies in the vertical plane through the
// source and that column.  In the view frame of the 3D kernel above, the x and
// y slab intervals of ray (u, v) in a voxel,
//   s in [(du e_u,k -+ h_k) / D~_k(u)],  k = x, y,  du = Bu - A u / sdd,
// depend on u and the voxel's column (A, Bu: view-frame coordinates of the
// column's centre) only, and its z slab interval
//   s in [(z_f - z_S) sdd / (e_v,z v) - A],  z_f = the voxel's two z faces,
// on v and the voxel only.  The clip length of a pair is therefore
//   |D~| max(0, min(X_hi(u), Z_hi(v)) - max(X_lo(u), Z_lo(v)))
// with X the column's xy interval of ray u and Z the voxel's z interval of row
// v: X is formed once per (column, u) and Z once per (voxel, v) instead of
// three slab intervals per pair.  A work-group owns NC voxel columns x TZ
// voxels in z (z fastest, col_vz voxels a lane; col_tile_shape) and walks the
// group's views in rounds of 256 / NC.  At the start of a round one lane per
// (view, column) forms the tile's detector window, the column's bins in it,
// X of its first two and the constants of its voxels' row ranges.  Per view
// the work-group stages in LDS the product |D~| r of every ray of the window
// and sdd / (e_v,z v) of every row (float64: the z bounds are differences of
// terms of the size of A); each voxel then takes the rows of its shadow and,
// per row, the bins of its column.  Both bounds are formed in float64 up to a
// difference, so they keep their precision for rays nearly parallel to a
// voxel face (the small direction components that the float32 bounds of the
// general kernel lose).  A zero direction component (the kernels' rule)
// keeps the ray in the source's slab of that axis.
constexpr int kColWG = 4;         // resident work-groups per CU the register budget is set for (128 VGPRs)
constexpr int kColR = 512;        // rays of a view's window staged at once (fast path: the whole window)
constexpr int kColV = 128;        // rows of a view's window staged at once
constexpr int kColU = 2;          // X intervals kept per (view, column); wider columns form the rest
constexpr int kColVZ = kColVoxels;  // voxels a lane at most (col_tile_shape)
constexpr int kColTiles = 512;    // a group's tiles listed in LDS (more: each round walks the entries)

// Per (view, column) of a round.
struct ColView {
    double A;                     // view-frame depth of the column's centre, times 2^colk_e
    float sm, sh;                 // mean and half difference of 1 / (A -+ half the footprint's depth
                                  // extent), over the row pitch
    float cl, ch;                 // centre row -+ margin (-+1e30 where the footprint reaches the source's depth)
    int32_t u0, u1;               // its bins within the tile's window
    int32_t co;                   // u0 - the window's first bin, clamped to [-2, window width - 1]
    int32_t rva;                  // co - v0 (window width): row k's rays from k (width) + rva
    float2 X[kColU];              // X of bins u0 and u0 + 1 (empty where absent)
};
// Per view of a round: the tile's detector window [u0, u1) x [v0, v1), whether
// it is staged whole (flag 1), whether the view has a zero component (2) and
// whether every voxel of the tile has at most two rows and every column at
// most two bins (4).
// A voxel at level l has f = sdd e_v,z (z - z_S) in [fl, fl + |svz|] with
// fl = f00 + l svz.
struct WinView {
    double zS;                    // source height
    float svz, f00;
    float fv0, fv1, dfl;          // v0 and v1 - 1 as floats; svz times the lanes of a column
    int32_t view, u0, u1, v0, v1, flags;
};

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float rflf(float v) { return __int_as_float(rfl(__float_as_int(v))); }
__device__ __forceinline__ double rfld(double v) {
    const long long b = __double_as_longlong(v);
    return __longlong_as_double(((long long)(unsigned)rfl((int)(b >> 32)) << 32) | (unsigned)rfl((int)b));
}

// The fields of a WinView that the staging needs, in scalar registers.
struct WinS {
    int view, u0, u1, v0, v1, flags;
};
__device__ __forceinline__ WinS win_s(const WinView& w) {
    return WinS{rfl(w.view), rfl(w.u0), rfl(w.u1), rfl(w.v0), rfl(w.v1), rfl(w.flags)};
}

// X of the ray of bin iu in the voxel column (jx, jy) whose centre has
// view-frame coordinates (A, B): the overlap of its x and y slab intervals
// (half widths hx, hy), with the bounds' numerators in float64.  dxy: the
// ray's float32 D~_x, D~_y; a zero component keeps the ray in the source's
// slab (skx, sky) of that axis.
__device__ __forceinline__ float2 col_interval(const DGeom& G, const double* V, const float2 dxy, double A,
                                               double B, int iu, int jx, int jy, int skx, int sky, double hx,
                                               double hy) {
    const double uu = ((double)iu - 0.5 * (double)(G.nu - 1)) * G.pu;
    const double du = fma(-A, uu * V[16], B);
    float lo = -INFINITY, hi = INFINITY;
    const float dk[2] = {dxy.x, dxy.y};
    const int ji[2] = {jx, jy}, sk[2] = {skx, sky};
    const double hk[2] = {hx, hy};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (fabsf(dk[k]) <= kAxisEpsF) {
            if (ji[k] != sk[k]) hi = -INFINITY;
        } else {
            const double num = du * V[6 + k];
            const float ik = __builtin_amdgcn_rcpf(dk[k]);
            const float p = (float)(num - hk[k]) * ik, q = (float)(num + hk[k]) * ik;
            lo = fmaxf(lo, fminf(p, q));
            hi = fminf(hi, fmaxf(p, q));
        }
    }
    return make_float2(lo, hi);
}

__device__ __forceinline__ float2 f4xy(const float4 q) { return make_float2(q.x, q.y); }

__device__ __forceinline__ int src_slab(double s, double o, double ih) {
    return (int)fmin(fmax(floor((s - o) * ih), -1e9), 1e9);
}

// The overlap of X and Z, at least 0: the intervals are scaled by 2^colk_e,
// so the overlap is at most 1 and the clamp to [0, 1] (an output modifier of
// the subtraction) is its lower bound alone.
__device__ __forceinline__ float col_clip(float2 X, float zl, float zh) {
    return __builtin_amdgcn_fmed3f(fminf(X.y, zh) - fmaxf(X.x, zl), 0.f, 1.f);
}

template <class BA>
__device__ __forceinline__ void back3c_body(const DGeom& G, const BA& a, const int gi, const int bt,
                                            const int n_tiles) {
    __shared__ ColView cv[256];                  // [view slot][column]
    __shared__ WinView wv[16];                   // [view slot] (at least 16 columns: at most 16 views a round)
    // |D~| r of a window's rays, two views in flight.  Two zero floats before
    // each buffer, and room after it for one more row of the widest window
    // (one row of kColR) and two floats, so that the two bins a voxel reads
    // per row, and the row after a staged part (zeroed by stage()), stay
    // inside it (the row loops below)
    __shared__ float sRb[2][2 * kColR + 4];
    // per row of a staged part: 2^e sdd / D_z (one more read, not used) and,
    // 8 KiB-apart in the same record so that one address serves both, the
    // float32 widths vz 2^e sdd / D_z of the row and the next (0 past the part)
    struct RowC {
        double isv[kColV + 1];
        float2 w[kColV + 1];
    };
    __shared__ RowC sI[2];
    __shared__ double zlev[32];                  // height of the lower face of each level of the tile
    // the group's tiles: view, u0 | u1 << 16, v0 | v1 << 16
    __shared__ int3 tix[kColTiles];
    __shared__ int wvote[4];                     // a wave's vote: some column not two rows, two bins
    __shared__ double sh[4];
    const int t = threadIdx.x;
    int TZ, CX, CY;
    col_tile_shape(a.box.z1 - a.box.z0, TZ, CX, CY);
    TZ = rfl(TZ);
    CX = rfl(CX);
    CY = rfl(CY);
    const int VZ = rfl(col_vz(TZ)), TL = rfl(TZ / VZ);     // voxels a lane, lanes a column
    const int NC = CX * CY, NVR = 256 / NC;                // columns; views per round
    // all four are powers of two: lane indices split with shifts and masks
    const int lgTL = __builtin_ctz(TL), lgNC = __builtin_ctz(NC), lgCX = __builtin_ctz(CX);
    const int tiles_x = a.tiles_x, tiles_y = a.tiles_y;
    const int tx = bt % tiles_x, ty = (bt / tiles_x) % tiles_y, tz = bt / (tiles_x * tiles_y);
    const int xs = a.box.x0 + tx * CX, ys = a.box.y0 + ty * CY, zs = a.box.z0 + tz * TZ;
    const int nvx = min(CX, a.box.x1 - xs), nvy = min(CY, a.box.y1 - ys), nvz = min(TZ, a.box.z1 - zs);
    // this lane's voxels: column c (cx, cy), levels lz, lz + TL, ...
    const int lz = t & (TL - 1), c = t >> lgTL;
    const int ccx = c & (CX - 1), ccy = c >> lgCX;
    const int ix = xs + ccx, iy = ys + ccy;
    const bool colv = ccx < nvx && ccy < nvy;
    bool valid[kColVZ];
#pragma unroll
    for (int q = 0; q < kColVZ; ++q) valid[q] = colv && q < VZ && lz + q * TL < nvz;
    // every value of sRb and sI is zero or one written by stage(): finite
    for (int i = t; i < 2 * (2 * kColR + 4); i += 256) (&sRb[0][0])[i] = 0.f;
    for (int i = t; i < 2 * (kColV + 1); i += 256) {
        sI[i / (kColV + 1)].isv[i % (kColV + 1)] = 0.0;
        sI[i / (kColV + 1)].w[i % (kColV + 1)] = make_float2(0.f, 0.f);
    }
    if (t < 32) zlev[t] = fma((double)(zs + t), G.vz, G.oz);

    int e0 = 0, e1 = a.n_ent;
    if (a.gptr) {
        e0 = a.gptr[gi];
        e1 = a.gptr[gi + 1];
    }
    int nt = 0;                                          // views (tiles) of the group
    for (int e = e0; e < e1; ++e) {
        const int rb = get_entry(a, e).rb;
        nt += G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
    }
    // the group's tiles, listed once in LDS (thread i finds tile i), so that a
    // round's set-up reads its tile, and loads its view, without walking the
    // entries or loading the tile (detectors of at most 65535 bins and rows)
    const bool listed = nt <= kColTiles && G.nu <= 65535 && G.nv <= 65535;
    if (listed) {
        for (int i = t; i < nt; i += 256) {
            int e = e0, off = i;
            for (;;) {
                const int rb = get_entry(a, e).rb;
                const int p0 = G.rb_tile_ptr[rb], cnt = G.rb_tile_ptr[rb + 1] - p0;
                if (off < cnt) {
                    const Tile tt = G.tiles[p0 + off];
                    tix[i] = make_int3(tt.view, tt.u0 | (tt.u1 << 16), tt.v0 | (tt.v1 << 16));
                    break;
                }
                off -= cnt;
                ++e;
            }
        }
    }
    __syncthreads();

    // rays [0, nr) (rows of pw bins from (ua, va)) and rows [0, nrow) of a
    // window part of `view` into buffer b
    auto stage = [&](int view, int b, int pw, int ua, int va, int nr, int nrow) {
        // the buffer index passes through an empty asm statement, so the
        // buffers' offsets are formed here rather than held across the views
        asm volatile("" : "+s"(b));
        const float* rview = a.r + (size_t)view * G.nv * G.nu;
        const float4* dxy = G.cdxy + (size_t)view * G.nu;
        const float* dz = G.cdz + (size_t)view * G.nv;
        // row of element i: (i + 1/2) / pw lies at least 1/(2 pw) from an
        // integer, far beyond the rounding of rcp and the product for i < 2^12
        const float ipw = __builtin_amdgcn_rcpf((float)pw);
        // a part holds at most 2 x 256 rays and 256 rows: each thread's two
        // rays and its row constants are loaded first, then written, so their
        // loads wait once
        static_assert(kColR <= 2 * 256 && kColV < 256, "two rays and one row a thread");
        const double* isv = G.cisv + (size_t)view * G.nv;
        float q2[2], z[2], rr[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = t + 256 * k;
            q2[k] = 0.f;
            z[k] = 0.f;
            rr[k] = 0.f;
            if (i < nr) {
                const int row = (int)(((float)i + 0.5f) * ipw);
                const int iu = ua + (i - __umul24(row, pw)), iv = va + row;
                q2[k] = ldu(reinterpret_cast<const float*>(dxy + iu), 2u);   // D~_x^2 + D~_y^2
                z[k] = ldu(dz, (unsigned)iv);
                rr[k] = ldu(rview, (unsigned)(iv * G.nu + iu));
            }
        }
        double s0 = 0.0, s1 = 0.0;
        if (t < nrow) {
            s0 = ldu(isv, (unsigned)(va + t));
            if (t + 1 < nrow) s1 = ldu(isv, (unsigned)(va + t + 1));
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = t + 256 * k;
            if (i < nr) sRb[b][2 + i] = __builtin_amdgcn_sqrtf(fmaf(z[k], z[k], q2[k])) * rr[k];
        }
        // the row after the part reads zeros (and two more floats)
        for (int i = t; i < pw + 2; i += 256) sRb[b][2 + nr + i] = 0.f;
        if (t < nrow) {
            sI[b].isv[t] = s0;
            sI[b].w[t] = make_float2((float)(G.vz * s0), (float)(G.vz * s1));
        }
    };

    float accv[kColVZ];
#pragma unroll
    for (int q = 0; q < kColVZ; ++q) accv[q] = 0.f;
    // this lane's voxels from a staged part of view j (buffer b, rows
    // [va, vb), bins [ua, ub) of pw a row).  FAST: the part is the whole
    // window, whose bins ColView already holds; CAREFUL: the view has a ray
    // with a zero direction component.
    auto both = [&](auto fast_c, auto careful_c, int j, const WinS& Ws, const ColView& C, int b, int pw, int ua,
                    int ub, int va, int vb) {
        constexpr bool FAST = decltype(fast_c)::value, CAREFUL = decltype(careful_c)::value;
        const float* R = &sRb[b][2];
        const double* SIv = sI[b].isv - va;              // row k at SIv[k]
        const double zS = wv[j].zS;
        const float svz = wv[j].svz, f00 = wv[j].f00, asvz = fabsf(svz);
        int rva = C.rva;
        float fva = wv[j].fv0, fvb = wv[j].fv1;
        const double A = C.A;
        const int cu0 = C.u0, cu1 = C.u1;
        float2 X0 = C.X[0], X1 = C.X[1];
        int co = C.co;
        int xu0 = cu0 + kColU, uH = cu1;
        if constexpr (!FAST) {
            // the part's bins: an absent bin gets an empty interval (clip 0;
            // the value it reads is not used)
            const int uL = max(cu0, ua);
            uH = min(cu1, ub - 1);
            if (!(cu0 >= uL && cu0 <= uH)) X0 = make_float2(INFINITY, -INFINITY);
            if (!(cu0 + 1 >= uL && cu0 + 1 <= uH)) X1 = make_float2(INFINITY, -INFINITY);
            // where the offset of bin cu0 lies outside [-2, pw - 1] neither
            // bin is in the part, and the clamped offset keeps the reads in
            // the buffer and its zero pads
            co = min(max(cu0 - ua, -2), pw - 1);
            xu0 = max(uL, cu0 + kColU);
            rva = co - __umul24(va, pw);
            fva = (float)va;
            fvb = (float)(vb - 1);
        }
        const bool wide = xu0 <= uH;
        const float sm = C.sm, sh = C.sh, cl = C.cl, ch = C.ch;
        // f of the lower face of the lane's voxel q, stepped by TL levels
        const float dfl = wv[j].dfl;
        float fl = fmaf((float)lz, svz, f00);
        int ssrc = 0;                                    // the source's level in the tile
        if constexpr (CAREFUL) ssrc = src_slab(zS, G.oz, G.ivz) - zs;
        if constexpr (FAST && !CAREFUL) {
            if (Ws.flags & 4) {
                // every voxel of the view has at most two rows and every
                // column at most two bins: rows k0 and k0 + 1 of every voxel
                // (as in the two-row branch below), the lane's voxels in one
                // straight run with no test, so that their reads of LDS are
                // issued together.  A voxel outside the box reads inside the
                // buffers (its row is clamped to the window, its column's
                // offset to the window's width) and its sum is dropped.
                // the lower face of voxel q over the source, stepped by TL
                // levels (the level passes through an empty asm statement, so
                // that the first is formed here rather than held across the views)
                int zl0 = zs + lz;
                asm volatile("" : "+v"(zl0));
                double zfl = fma((double)zl0, G.vz, rfld(G.oz - zS));
                const double dzq = (double)TL * G.vz;
                // byte addresses: row k's first ray at Rb - 4 pw nk, its row
                // constants at Sb - 8 nk (nk = -k, the negated ceiling being a
                // floor of the negation)
                const char* Rb = reinterpret_cast<const char*>(R) + 4 * rva;
                const char* Sb = reinterpret_cast<const char*>(sI[b].isv);
                const int m4pw = -4 * pw;
                const float fnv0 = (float)(-va), fnv1 = (float)(1 - vb);
#pragma unroll
                for (int q = 0; q < kColVZ; ++q) {
                    if (q > 0) {
                        fl += dfl;
                        zfl += dzq;
                    }
                    const float lo = fmaf(-fabsf(fl), sh, fmaf(fl, sm, cl));
                    // -k0, k0 = ceil(lo) clamped to the window's rows (the
                    // clamp to integer bounds commutes with the floor)
                    const int nk = (int)floorf(__builtin_amdgcn_fmed3f(-lo, fnv1, fnv0));
                    const char* ra = Rb + __mul24(nk, m4pw);
                    const char* sa = Sb + __mul24(nk, -8) - 8 * va;
                    // the row constants and the four rays, read together
                    const double iA = *reinterpret_cast<const double*>(sa);
                    const double iB = *reinterpret_cast<const double*>(sa + 8);
                    const float2 wAB = *reinterpret_cast<const float2*>(sa + offsetof(RowC, w));
                    const float r0 = *reinterpret_cast<const float*>(ra);
                    const float r1 = *reinterpret_cast<const float*>(ra + 4);
                    const float r2 = *reinterpret_cast<const float*>(ra + 4 * pw);
                    const float r3 = *reinterpret_cast<const float*>(ra + 4 * pw + 4);
                    const float pfA = (float)fma(zfl, iA, -A), pfB = (float)fma(zfl, iB, -A);
                    const float rfA = pfA + wAB.x, rfB = pfB + wAB.y;
                    const float zlA = fminf(pfA, rfA), zhA = fmaxf(pfA, rfA);
                    const float zlB = fminf(pfB, rfB), zhB = fmaxf(pfB, rfB);
                    float acc = accv[q];
                    acc = fmaf(col_clip(X0, zlA, zhA), r0, acc);
                    acc = fmaf(col_clip(X1, zlA, zhA), r1, acc);
                    acc = fmaf(col_clip(X0, zlB, zhB), r2, acc);
                    acc = fmaf(col_clip(X1, zlB, zhB), r3, acc);
                    accv[q] = acc;
                }
                return;
            }
        }
#pragma unroll
        for (int q = 0; q < kColVZ; ++q) {
            if (q > 0) fl += dfl;
            if (!valid[q]) continue;
            // rows of the voxel: v = f / A' over the depths A' of its column's
            // footprint, f over its two faces: [f sm - |f| sh, f sm + |f| sh]
            // is f over the two depths
            const float fh = fl + asvz;
            const float lo = fmaf(-fabsf(fl), sh, fmaf(fl, sm, cl));
            const float hi = fmaf(fabsf(fh), sh, fmaf(fh, sm, ch));
            const int k0 = (int)__builtin_amdgcn_fmed3f(ceilf(lo), fva, fvb), k1 = (int)fminf(floorf(hi), fvb);
            // the voxel's lower face over the source
            const double zfl = zlev[lz + q * TL] - zS;
            bool in_src = false;
            if constexpr (CAREFUL) in_src = lz == ssrc - q * TL;
            auto zint = [&](double isv, float& zl, float& zh) {
                if (CAREFUL && isv == 0.0) {
                    // a horizontal ray stays at the source's height
                    zl = in_src ? -INFINITY : INFINITY;
                    zh = in_src ? INFINITY : -INFINITY;
                } else {
                    const double p = fma(zfl, isv, -A);
                    const float pf = (float)p, rf = (float)fma(G.vz, isv, p);
                    zl = fminf(pf, rf);
                    zh = fmaxf(pf, rf);
                }
            };
            float acc = accv[q];
            if ((FAST && (Ws.flags & 4)) || __all(k1 - k0 <= 1 && !wide)) {
                // at most two rows in every lane (the usual case): rows k0
                // and k0 + 1 without a loop.  A row outside [k0, k1] misses
                // the voxel by more than the row range's margin (1e-3 of a
                // row), far beyond rounding, so its clips are exactly 0; row
                // k0 + 1 may be one past the part, whose rays the staging
                // left zero (its row constant, read from the pad, is not
                // used).
                float zlA, zhA, zlB, zhB;
                zint(SIv[k0], zlA, zhA);
                zint(SIv[k0 + 1], zlB, zhB);
                const int rA = __umul24(k0, pw) + rva, rB = rA + pw;
                acc = fmaf(col_clip(X0, zlA, zhA), R[rA], acc);
                acc = fmaf(col_clip(X1, zlA, zhA), R[rA + 1], acc);
                acc = fmaf(col_clip(X0, zlB, zhB), R[rB], acc);
                acc = fmaf(col_clip(X1, zlB, zhB), R[rB + 1], acc);
            } else {
                int rb = __umul24(k0, pw) + rva - co;
                for (int k = k0; k <= k1; ++k, rb += pw) {
                    float zl, zh;
                    zint(SIv[k], zl, zh);
                    acc = fmaf(col_clip(X0, zl, zh), R[rb + co], acc);
                    acc = fmaf(col_clip(X1, zl, zh), R[rb + co + 1], acc);
                    if (wide) {
                        // a column more than kColU bins wide: X of the rest formed here
                        const int view = rfl(wv[j].view);
                        const double* V = view_of(G, view);
                        int wix = ix, wiy = iy;
                        asm volatile("" : "+v"(wix), "+v"(wiy));
                        const double qx = G.ox + ((double)wix + 0.5) * G.vx - V[0];
                        const double qy = G.oy + ((double)wiy + 0.5) * G.vy - V[1];
                        const double A0 = fma(qx, V[12], qy * V[13]);
                        for (int u = xu0; u <= uH; ++u) {
                            const float2 xi = col_interval(G, V, f4xy(ldu(G.cdxy + (size_t)view * G.nu, (unsigned)u)), A0,
                                                           fma(qx, V[6], qy * V[7]), u, ix, iy,
                                                           src_slab(V[0], G.ox, G.ivx), src_slab(V[1], G.oy, G.ivy),
                                                           0.5 * G.vx, 0.5 * G.vy);
                            acc = fmaf(col_clip(make_float2(ldexpf(xi.x, G.colk_e), ldexpf(xi.y, G.colk_e)), zl, zh),
                                       R[rb + (u - ua)], acc);
                        }
                    }
                }
            }
            accv[q] = acc;
        }
    };
    auto both_u = [&](auto fast_c, int j, const WinS& W, int b, int pw, int ua, int ub, int va, int vb) {
        // the lane's column index passes through an empty asm statement, so
        // its slot's address is formed per view rather than held
        int cc = c;
        asm volatile("" : "+v"(cc));
        const ColView& C = cv[j * NC + cc];
        if (W.flags & 2)
            both(fast_c, std::true_type{}, j, W, C, b, pw, ua, ub, va, vb);
        else
            both(fast_c, std::false_type{}, j, W, C, b, pw, ua, ub, va, vb);
    };

    for (int base = 0; base < nt; base += NVR) {
        const int nvr = min(NVR, nt - base);
        // phase A: lane (view slot j, column cc) of the round.  The tile's
        // corner and extent pass through an empty asm statement, so that the
        // float64 terms formed from them stay in this loop instead of being
        // held in registers across it (more than the budget holds)
        {
            int pt = t, pxs = xs, pys = ys, pzs = zs, pnx = nvx, pny = nvy, pnz = nvz, pnv = G.nv;
            double ppv = G.pv, phx = G.vx, phy = G.vy;
            asm volatile("" : "+v"(pt), "+s"(pxs), "+s"(pys), "+s"(pzs), "+s"(pnx), "+s"(pny), "+s"(pnz), "+s"(pnv));
            asm volatile("" : "+s"(ppv), "+s"(phx), "+s"(phy));
            const float fc0v = (float)(0.5 * (double)(pnv - 1)), ipv = (float)(1.0 / ppv);
            phx *= 0.5;
            phy *= 0.5;
            const int j = pt >> lgNC, cc = pt & (NC - 1);
            if (j < nvr) {
                Tile tl{};
                if (listed) {
                    const int3 tc = tix[base + j];
                    tl = Tile{tc.x, tc.y & 0xffff, (int)((unsigned)tc.y >> 16), tc.z & 0xffff,
                              (int)((unsigned)tc.z >> 16)};
                } else {
                    int e = e0, off = base + j;
                    for (;;) {
                        const int rb = get_entry(a, e).rb;
                        const int cnt = G.rb_tile_ptr[rb + 1] - G.rb_tile_ptr[rb];
                        if (off < cnt) {
                            tl = G.tiles[G.rb_tile_ptr[rb] + off];
                            break;
                        }
                        off -= cnt;
                        ++e;
                    }
                }
                const double* V = view_of(G, tl.view);
                const double sdd = V[15];
                const double c0u = 0.5 * (double)(G.nu - 1);
                const float su = (float)(sdd / G.pu), fu = (float)c0u;
                // the tile's window: the projections of its box's corners (every
                // lane of the view slot forms it; its column lane 0 stores it)
                const double ssv = sdd * V[11];
                int wu0 = tl.u0, wu1 = tl.u1, wv0 = tl.v0, wv1 = tl.v1;
                {
                    const double x0 = G.ox + (double)pxs * G.vx - V[0], y0 = G.oy + (double)pys * G.vy - V[1];
                    const double z0 = G.oz + (double)pzs * G.vz - V[2];
                    const float ex = (float)V[6], ey = (float)V[7], nx = (float)V[12], ny = (float)V[13];
                    const float xa = (float)x0, xb = (float)(x0 + pnx * G.vx);
                    const float ya = (float)y0, yb = (float)(y0 + pny * G.vy);
                    const float za = (float)z0, zb = (float)(z0 + pnz * G.vz);
                    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
                    bool front = true;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float px = (k & 1) ? xb : xa, py = (k & 2) ? yb : ya;
                        const float Ak = fmaf(py, ny, px * nx);
                        front = front && Ak > 0.f;
                        const float iA = __builtin_amdgcn_rcpf(Ak);
                        const float uu = fmaf(py, ey, px * ex) * iA;
                        umin = fminf(umin, uu);
                        umax = fmaxf(umax, uu);
                        vmin = fminf(vmin, fminf(za * iA, zb * iA));
                        vmax = fmaxf(vmax, fmaxf(za * iA, zb * iA));
                    }
                    if (front) {
                        const float bl = fmaf(umin, su, fu), bh = fmaf(umax, su, fu);
                        wu0 = max(wu0, (int)ceilf(bl - 1e-3f - 1e-6f * fabsf(bl)));
                        wu1 = min(wu1, (int)floorf(bh + 1e-3f + 1e-6f * fabsf(bh)) + 1);
                        // v = sdd e_v,z (z - z_S) / A: scale the extremes by ssv
                        const float sv = (float)ssv * ipv;
                        const float cl = fminf(vmin * sv, vmax * sv) + fc0v, ch = fmaxf(vmin * sv, vmax * sv) + fc0v;
                        wv0 = max(wv0, (int)ceilf(cl - 1e-3f - 1e-6f * fabsf(cl)));
                        wv1 = min(wv1, (int)floorf(ch + 1e-3f + 1e-6f * fabsf(ch)) + 1);
                    }
                    wu1 = max(wu0, wu1);
                    wv1 = max(wv0, wv1);
                    if (cc == 0) {
                        WinView& W = wv[j];
                        W.view = tl.view;
                        W.zS = V[2];
                        const double svz = ssv * G.vz;
                        W.svz = (float)svz;
                        // the lower f of the two faces of level 0
                        W.f00 = (float)(ssv * (G.oz + (double)pzs * G.vz - V[2]) + fmin(svz, 0.0));
                        W.u0 = wu0;
                        W.u1 = wu1;
                        W.v0 = wv0;
                        W.v1 = wv1;
                        W.fv0 = (float)wv0;
                        W.fv1 = (float)(wv1 - 1);
                        W.dfl = (float)TL * (float)svz;
                        const bool fast = (wu1 - wu0) * (wv1 - wv0) <= kColR && wv1 - wv0 <= kColV;
                        W.flags = (fast ? 1 : 0) | ((G.view_flags[tl.view] & 1) ? 2 : 0);
                    }
                }
                // the column
                const int jx = pxs + (cc & (CX - 1)), jy = pys + (cc >> lgCX);
                const double qx = G.ox + ((double)jx + 0.5) * G.vx - V[0];
                const double qy = G.oy + ((double)jy + 0.5) * G.vy - V[1];
                const double A = fma(qx, V[12], qy * V[13]);
                const double B = fma(qx, V[6], qy * V[7]);
                const double ea = phx * fabs(V[12]) + phy * fabs(V[13]);
                ColView& C = cv[pt];
                C.A = ldexp(A, G.colk_e);                       // the scale of the intervals
                const bool ok = A - ea > 0.0;
                // row ranges: v = f / A' / pv + c0v over A' in [A - ea, A + ea];
                // a footprint at the source's depth takes every row
                const float mrg = 1e-3f + 1e-6f * (float)pnv;
                const float sl0 = ok ? __builtin_amdgcn_rcpf((float)(A - ea)) * ipv : 0.f;
                const float sl1 = ok ? __builtin_amdgcn_rcpf((float)(A + ea)) * ipv : 0.f;
                C.sm = 0.5f * (sl0 + sl1);
                C.sh = 0.5f * (sl0 - sl1);
                C.cl = ok ? fc0v - mrg : -1e30f;
                C.ch = ok ? fc0v + mrg : 1e30f;
                // bins in the window whose ray can meet the column: the
                // projections of its footprint's corners (it lies in front of
                // the source)
                int u0 = wu0, u1 = wu1 - 1;
                if (ok) {
                    const float hxf = (float)phx, hyf = (float)phy;
                    const float Af = (float)A, Bf = (float)B;
                    const float nx = (float)V[12], ny = (float)V[13], ex = (float)V[6], ey = (float)V[7];
                    float umin = INFINITY, umax = -INFINITY;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float px = (k & 1) ? hxf : -hxf, py = (k & 2) ? hyf : -hyf;
                        const float uu = fmaf(py, ey, fmaf(px, ex, Bf)) *
                                         __builtin_amdgcn_rcpf(fmaf(py, ny, fmaf(px, nx, Af)));
                        umin = fminf(umin, uu);
                        umax = fmaxf(umax, uu);
                    }
                    const float bl = fmaf(umin, su, fu), bh = fmaf(umax, su, fu);
                    u0 = max(u0, (int)ceilf(bl - 1e-3f - 1e-6f * fabsf(bl)));
                    u1 = min(u1, (int)floorf(bh + 1e-3f + 1e-6f * fabsf(bh)));
                }
                C.u0 = u0;
                C.u1 = u1;
                C.co = min(u0 - wu0, max(1, wu1 - wu0) - 1);    // u0 >= wu0
                C.rva = C.co - wv0 * max(1, wu1 - wu0);
                // at most two bins, and at most two rows at every level: the
                // rows of a voxel span hi - lo = fh s - fl s' + (ch - cl),
                // which is convex in the level, so its largest value is at the
                // lowest or the highest level; below 1.9 (not 2: the voxels
                // round their own bounds) it leaves room for two integers
                bool simple = u1 <= u0 + 1 && ok;
                {
                    const float svz = (float)(ssv * G.vz), asvz = fabsf(svz);
                    const float f00 = (float)(ssv * (G.oz + (double)pzs * G.vz - V[2]) + fmin(ssv * G.vz, 0.0));
#pragma unroll
                    for (int e2 = 0; e2 < 2; ++e2) {
                        const float fl = fmaf((float)(e2 ? pnz - 1 : 0), svz, f00), fh = fl + asvz;
                        const float lo = fl * (fl >= 0.f ? sl1 : sl0) + C.cl;
                        const float hi = fh * (fh >= 0.f ? sl0 : sl1) + C.ch;
                        simple = simple && hi - lo < 1.9f;
                    }
                }
                // where the view slot's NC lanes lie in one wave (NC <= 64, a
                // power of two) its column lane 0 sets the flag; else (the
                // slot spans NC / 64 whole waves) each wave leaves its vote
                // for the slot's waves to be combined after the barrier
                const unsigned long long bal = __ballot(!simple);
                if (NC <= 64) {
                    const unsigned long long slot = (NC == 64 ? ~0ull : ((1ull << NC) - 1ull))
                                                    << ((pt & 63) & ~(NC - 1));
                    if (cc == 0 && (bal & slot) == 0ull) wv[j].flags |= 4;
                } else if ((pt & 63) == 0) {
                    wvote[pt >> 6] = bal != 0ull ? 1 : 0;
                }
                const int skx = src_slab(V[0], G.ox, G.ivx), sky = src_slab(V[1], G.oy, G.ivy);
#pragma unroll
                for (int i = 0; i < kColU; ++i) {
                    const int u = u0 + i;
                    float2 xi = make_float2(INFINITY, -INFINITY);
                    if (u <= u1) {
                        xi = col_interval(G, V, f4xy(ldu(G.cdxy + (size_t)tl.view * G.nu, (unsigned)u)), A, B, u, jx, jy,
                                          skx, sky, phx, phy);
                        xi.x = ldexpf(xi.x, G.colk_e);
                        xi.y = ldexpf(xi.y, G.colk_e);
                    }
                    C.X[i] = xi;
                }
            }
        }
        __syncthreads();
        if (NC > 64) {
            // a view slot of NC / 64 waves: two rows and two bins where none
            // of its waves voted otherwise
            if (t < nvr) {
                const int wps = NC >> 6;
                bool any = false;
                for (int w = t * wps; w < (t + 1) * wps; ++w) any = any || wvote[w] != 0;
                if (!any) wv[t].flags |= 4;
            }
            __syncthreads();
        }
        // the round's views, one barrier each: the next view's window is staged
        // while this one's is gathered
        WinS W = win_s(wv[0]);
        if (W.flags & 1)
            stage(W.view, 0, max(1, W.u1 - W.u0), W.u0, W.v0, (W.u1 - W.u0) * (W.v1 - W.v0), W.v1 - W.v0);
        __syncthreads();
        for (int j = 0; j < nvr; ++j) {
            const int b = j & 1;
            const bool more = j + 1 < nvr;
            const WinS Wn = win_s(wv[min(j + 1, nvr - 1)]);
            const bool empty = W.u1 <= W.u0 || W.v1 <= W.v0;
            if (W.flags & 1) {
                if (more && (Wn.flags & 1))
                    stage(Wn.view, b ^ 1, max(1, Wn.u1 - Wn.u0), Wn.u0, Wn.v0, (Wn.u1 - Wn.u0) * (Wn.v1 - Wn.v0),
                          Wn.v1 - Wn.v0);
                if (!empty)
                    both_u(std::true_type{}, j, W, b, max(1, W.u1 - W.u0), W.u0, W.u1, W.v0, W.v1);
                __syncthreads();
            } else {
                // a window too large to stage whole: parts of at most kColR
                // rays and kColV rows, each between two barriers
                const int pw = max(1, W.u1 - W.u0), ppw = min(pw, kColR);
                for (int ua = W.u0; ua < W.u1; ua += ppw) {
                    const int ub = min(W.u1, ua + ppw), qw = ub - ua;
                    const int rows = max(1, min(kColV, kColR / qw));
                    for (int va = W.v0; va < W.v1; va += rows) {
                        const int vb = min(W.v1, va + rows);
                        __syncthreads();
                        stage(W.view, 0, qw, ua, va, qw * (vb - va), vb - va);
                        __syncthreads();
                        both_u(std::false_type{}, j, W, 0, qw, ua, ub, va, vb);
                    }
                }
                __syncthreads();
                if (more && (Wn.flags & 1)) {
                    stage(Wn.view, b ^ 1, max(1, Wn.u1 - Wn.u0), Wn.u0, Wn.v0, (Wn.u1 - Wn.u0) * (Wn.v1 - Wn.v0),
                          Wn.v1 - Wn.v0);
                    __syncthreads();
                }
            }
            W = Wn;
        }
    }

    const int nxJ = a.box.x1 - a.box.x0, nyJ = a.box.y1 - a.box.y0, nzJ = a.box.z1 - a.box.z0;
    double p = 0.0;
#pragma unroll
    for (int q = 0; q < kColVZ; ++q) {
        const float acc = ldexpf(accv[q], -G.colk_e);  // exact
        const int iz = zs + lz + q * TL;
        const size_t gix = ((size_t)iz * G.ny + iy) * G.nx + ix;
        if (!valid[q]) continue;
        if (a.fused) {
            const int jx = ix - a.box.x0, jy = iy - a.box.y0, jz = iz - a.box.z0;
            const float2 v = make_float2(a.x[gix], acc);
            float2* basep = a.xg + (size_t)gi * a.xg_stride + xg_pad(nxJ, nyJ, nzJ);
            basep[(jz * nyJ + jy) * nxJ + jx] = v;
            basep[xg_copy(nxJ, nyJ, nzJ) + (jz * nxJ + jx) * nyJ + jy] = v;
            p += (double)acc * (double)acc;
        } else {
            a.g[gix] = (a.flags & 1) ? a.g[gix] + acc : acc;
        }
    }
    if (a.fused) {
        const double tsum = block_sum256(p, sh);
        if (threadIdx.x == 0) a.partial[(size_t)gi * n_tiles + bt] = tsum;
    }
}

// The standalone products (entries inline in the arguments: more scalar
// registers) get the register budget of four work-groups per CU, where they
// need no scratch; the solver's launches keep kColWG.
template <class BA>
__global__ __launch_bounds__(256, BA::kInl ? 4 : kColWG) void k_back3c(DGeom G, BA a) {
    back3c_body(G, a, blockIdx.y, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------
// K3: step sizes mu = beta ||g||^2 / ||A g||^2 (Eq. 11, relaxed), one
// work-group per group, fixed-order float64 sums of the partials
// ----------------------------------------------------------------------------
__device__ __forceinline__ void step_body(const StepArgs& s, const int g, const int n_groups) {
    __shared__ double sh[4];
    // both sums' partials are read in one pass (they were written by other
    // XCDs, so each round trip costs a memory latency); each lane still adds
    // its elements of each sum in the same order
    const int c0 = s.ent[s.gptr[g]].chunk_prefix;
    const int c1 = (g + 1 < n_groups) ? s.ent[s.gptr[g + 1]].chunk_prefix : s.n_chunks;
    const int t0 = g * s.n_tiles, t1 = (g + 1) * s.n_tiles;
    double vg = 0.0, vq = 0.0;
    const int ng = t1 - t0, nq = c1 - c0;
    // four rounds of loads in flight at once, added in the same order
    constexpr int R = 4;
    for (int k0 = (int)threadIdx.x; k0 < max(ng, nq); k0 += R * 256) {
        double a[R], b[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int k = k0 + q * 256;
            a[q] = k < ng ? s.pg[t0 + k] : 0.0;
            b[q] = k < nq ? s.pq[c0 + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int k = k0 + q * 256;
            if (k < ng) vg += a[q];
            if (k < nq) vq += b[q];
        }
    }
    const double gg = block_sum256(vg, sh);
    __syncthreads();
    const double qq = block_sum256(vq, sh);
    if (threadIdx.x == 0) s.mu[g] = (gg > 0.0 && qq > 0.0) ? s.beta[g] * gg / qq : 0.0;
}

__global__ __launch_bounds__(256) void k_step(StepArgs s) { step_body(s, blockIdx.x, gridDim.x); }

// ----------------------------------------------------------------------------
// K4: finalize a column-block step
// ----------------------------------------------------------------------------

// sum_{j < n} z[j * M + ray] in ascending j, eight loads in flight at once
__device__ __forceinline__ float col_sum(const float* z, const int64_t M, const int n, const int ray) {
    float s = 0.f;
    for (int j0 = 0; j0 < n; j0 += 8) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = j0 + q < n ? z[(size_t)(j0 + q) * M + ray] : 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (j0 + q < n) s += v[q];
    }
    return s;
}

__device__ __forceinline__ void fin_body(const DGeom& G, const FinArgs& f, const int bid) {
    const int ray_blocks = (f.n_chunks + 3) / 4;
    if (bid < ray_blocks) {
        const int c = bid * 4 + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if (c >= f.n_chunks) return;
        const int ei = find_entry(f, c);
        const Entry en = get_entry(f, ei);
        const Chunk ch = chunk_of(G, en, c, 1, f.col);
        if (lane >= ch.cnt) return;
        const int k = ch.k0 + lane;
        const int ray = (ch.view * G.nv + ch.v0 + k / ch.w) * G.nu + ch.u0 + k % ch.w;
        const float mu = (float)f.mu[en.group];
        const float zn = fmaf(mu, f.q[en.slot_prefix + ch.roff + lane], f.zJ[ray]);
        f.zJ[ray] = zn;
        if (f.refresh) f.r[ray] = f.y[ray] - col_sum(f.z, f.M, f.n_cols, ray);
    } else {
        const int v = (bid - ray_blocks) * 256 + threadIdx.x;
        if (v >= f.vox_J) return;
        const int nxJ = f.box.x1 - f.box.x0, nyJ = f.box.y1 - f.box.y0;
        const int lx = v % nxJ, ly = (v / nxJ) % nyJ, lz = v / (nxJ * nyJ);
        const int nzJ = f.box.z1 - f.box.z0;
        const int li = xg_pad(nxJ, nyJ, nzJ) + v;           // copy 0 is x-fastest
        // the groups' pairs, four loads in flight at once, added in group order
        float s = 0.f;
        for (int g0 = 0; g0 < f.n_groups; g0 += 4) {
            float2 p[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                p[q] = g0 + q < f.n_groups ? f.xg[(size_t)(g0 + q) * f.xg_stride + li] : make_float2(0.f, 0.f);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (g0 + q < f.n_groups) s += fmaf((float)f.mu[g0 + q], p[q].y, p[q].x);
        }
        const size_t gix = ((size_t)(f.box.z0 + lz) * f.ny + (f.box.y0 + ly)) * f.nx + f.box.x0 + lx;
        f.x[gix] = s / (float)f.n_groups;
        if (G.mixed_boxes) {
            // Column blocks of unequal sizes lay their (x, g) copies out
            // differently, so this step's pairs could lie in the padding of a
            // later step's copies.  The forward walks read padding only for
            // segments that are zero up to float32 rounding; clearing both
            // copies here keeps the whole buffer zero between steps, so that
            // each step is a function of x, z and r alone.
            const int li1 = xg_copy(nxJ, nyJ, nzJ) + xg_pad(nxJ, nyJ, nzJ) + (lz * nxJ + lx) * nyJ + ly;
            for (int g = 0; g < f.n_groups; ++g) {
                float2* slot = f.xg + (size_t)g * f.xg_stride;
                slot[li] = make_float2(0.f, 0.f);
                slot[li1] = make_float2(0.f, 0.f);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_finalize(DGeom G, FinArgs f) { fin_body(G, f, blockIdx.x); }

// ----------------------------------------------------------------------------
// K5: residual refresh over the rays of a list of row blocks
// ----------------------------------------------------------------------------

__device__ __forceinline__ void res_body(const DGeom& G, const ResArgs& a, const int bid,
                                         const int n_chunks) {
    const int c = bid * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= n_chunks) return;
    const int ei = find_entry(a, c);
    const Entry en = get_entry(a, ei);
    const Chunk ch = chunk_of(G, en, c, 0, 0);
    if (lane >= ch.cnt) return;
    const int k = ch.k0 + lane;
    const int ray = (ch.view * G.nv + ch.v0 + k / ch.w) * G.nu + ch.u0 + k % ch.w;
    a.r[ray] = a.y[ray] - col_sum(a.z, a.M, a.n_cols, ray);
}

__global__ __launch_bounds__(256) void k_residual(DGeom G, ResArgs a, int n_chunks) {
    res_body(G, a, blockIdx.x, n_chunks);
}

// ----------------------------------------------------------------------------
// batched phases: one launch advances the same phase of every job of a batch.
// Each work-group finds its job from the per-job work-group prefix, rebuilds
// that job's launch arguments from the device job table and the job's own
// epoch counter, and runs the same body as the single-job kernel, so a job's
// results are the same bits in a batch as alone.
// ----------------------------------------------------------------------------
// Read a launch-constant table entry (job table, schedule records, boxes,
// epoch counters outside kb_advance) through the constant address space, so
// that wave-uniform reads become scalar loads into scalar registers.
template <class T>
__device__ __forceinline__ T cld(const T* p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    using CT = const __attribute__((address_space(4))) T*;
    return ((CT)p)[i];
#else
    return p[i];        // host pass: never executed
#endif
}

// Owner of work-group b: the last k with prefix[k] <= b (prefix is
// non-decreasing, so jobs without work in this phase are skipped).  Every
// lane of the wave must be active.
__device__ __forceinline__ int batch_job(const BatchArgs& B, const int b) {
    int cnt = 0;
    for (int base = 0; base < B.n_jobs; base += 64) {
        const int i = base + (int)(threadIdx.x & 63);
        const bool le = i < B.n_jobs && ldu(B.prefix, (unsigned)i) <= b;
        cnt += __popcll(__ballot(le));
    }
    return __builtin_amdgcn_readfirstlane(cnt - 1);
}

// Step c of job k's current epoch; false once the job has run all its epochs
// or its epoch has fewer steps.
__device__ __forceinline__ bool batch_step(const BatchArgs& B, const int k, const BJob& J, StepRec& sr) {
    const int e = cld(B.ep, k);
    if (e < 0 || e >= J.n_epochs) return false;
    const EpochRec er = cld(J.epochs, e);
    if (B.c >= er.n_steps) return false;
    sr = cld(J.steps, er.step0 + B.c);
    return sr.n_groups > 0;            // a column without groups is skipped, as alone
}

__device__ __forceinline__ void box_tiles(const Box& b, const int dims, const int vertical, int& tx, int& ty,
                                          int& tz) {
    if (dims == 2) {
        tx = (b.x1 - b.x0 + kTile2 - 1) / kTile2;
        ty = (b.y1 - b.y0 + kTile2 - 1) / kTile2;
        tz = 1;
    } else if (vertical) {
        int TZ, CX, CY;
        col_tile_shape(b.z1 - b.z0, TZ, CX, CY);
        tx = (b.x1 - b.x0 + CX - 1) / CX;
        ty = (b.y1 - b.y0 + CY - 1) / CY;
        tz = (b.z1 - b.z0 + TZ - 1) / TZ;
    } else {
        tx = (b.x1 - b.x0 + kTile3x - 1) / kTile3x;
        ty = (b.y1 - b.y0 + kTile3y - 1) / kTile3y;
        tz = (b.z1 - b.z0 + kTile3z - 1) / kTile3z;
    }
}

__device__ __forceinline__ int box_vox(const Box& b) {
    return (b.x1 - b.x0) * (b.y1 - b.y0) * (b.z1 - b.z0);
}

// occupancy as the single-job kernels: eight waves per SIMD in 2D, six in 3D;
// NW waves per 2D tile (the 3D tile always takes four)
template <int KIND, int NW>
__global__ __launch_bounds__(64 * NW, KIND == kCone ? 6 : (KIND == kConeV ? kColWG : back2_waves(NW, false))) void kb_back(BatchArgs B) {
    const int k = batch_job(B, blockIdx.x);
    const int L = blockIdx.x - B.prefix[k];
    const BJob J = cld(B.jobs, k);
    StepRec sr;
    if (!batch_step(B, k, J, sr)) return;
    const DGeom G = J.G;
    BackCore a{};
    a.box = cld(J.boxes, sr.col);
    box_tiles(a.box, G.dims, G.vertical, a.tiles_x, a.tiles_y, a.tiles_z);
    const int nt = a.tiles_x * a.tiles_y * a.tiles_z;
    const int gi = L / nt, tile = L - gi * nt;
    if (gi >= sr.n_groups) return;
    a.ent = J.ent + sr.ent_off;
    a.gptr = J.gptr + sr.gptr_off;
    a.n_ent = sr.n_ent;
    a.fused = 1;
    a.r = J.r;
    a.x = J.x;
    a.xg = J.xg;
    a.vox_J = box_vox(a.box);
    a.xg_stride = xg_size(a.box.x1 - a.box.x0, a.box.y1 - a.box.y0, a.box.z1 - a.box.z0);
    a.partial = J.pg;
    if constexpr (KIND == kConeV) back3c_body(G, a, gi, tile, nt);
    else if constexpr (KIND == kCone) back3_body(G, a, gi, tile, nt);
    else back2_body<KIND, BackCore, NW>(G, a, gi, tile, nt);
}

template <int KIND, int KS>
__global__ __launch_bounds__(256) void kb_fwd(BatchArgs B) {
    const int k = batch_job(B, blockIdx.x);
    const int L = blockIdx.x - B.prefix[k];
    const BJob J = cld(B.jobs, k);
    StepRec sr;
    if (!batch_step(B, k, J, sr)) return;
    if (L >= sr.n_chunks) return;
    const DGeom G = J.G;
    FwdCore a{};
    a.box = cld(J.boxes, sr.col);
    a.ent = J.ent + sr.ent_off;
    a.n_ent = sr.n_ent;
    a.n_chunks = sr.n_chunks;
    a.mode = 1;
    a.windowed = 1;
    a.col = sr.col;
    a.xg = J.xg;
    a.vox_J = box_vox(a.box);
    a.xg_stride = xg_size(a.box.x1 - a.box.x0, a.box.y1 - a.box.y0, a.box.z1 - a.box.z0);
    a.out = J.z + (size_t)sr.col * (size_t)J.M;
    a.q = J.q;
    a.partial = J.pq;
    fwd_body<KIND, 1, FwdCore, KS>(G, a, L);
}

__global__ __launch_bounds__(256) void kb_step(BatchArgs B) {
    const int k = batch_job(B, blockIdx.x);
    const int L = blockIdx.x - B.prefix[k];
    const BJob J = cld(B.jobs, k);
    StepRec sr;
    if (!batch_step(B, k, J, sr)) return;
    if (L >= sr.n_groups) return;
    const Box box = cld(J.boxes, sr.col);
    int tx, ty, tz;
    box_tiles(box, J.G.dims, J.G.vertical, tx, ty, tz);
    StepArgs a{};
    a.ent = J.ent + sr.ent_off;
    a.gptr = J.gptr + sr.gptr_off;
    a.n_chunks = sr.n_chunks;
    a.n_tiles = tx * ty * tz;
    a.pg = J.pg;
    a.pq = J.pq;
    a.beta = J.beta + sr.beta_off;
    a.mu = J.mu;
    step_body(a, L, sr.n_groups);
}

__global__ __launch_bounds__(256) void kb_finalize(BatchArgs B) {
    const int k = batch_job(B, blockIdx.x);
    const int L = blockIdx.x - B.prefix[k];
    const BJob J = cld(B.jobs, k);
    StepRec sr;
    if (!batch_step(B, k, J, sr)) return;
    const Box box = cld(J.boxes, sr.col);
    const int vox = box_vox(box);
    if (L >= (sr.n_chunks + 3) / 4 + (vox + 255) / 256) return;
    const DGeom G = J.G;
    FinArgs f{};
    f.ent = J.ent + sr.ent_off;
    f.n_ent = sr.n_ent;
    f.n_chunks = sr.n_chunks;
    f.mu = J.mu;
    f.q = J.q;
    f.z = J.z;
    f.zJ = J.z + (size_t)sr.col * (size_t)J.M;
    f.y = J.y;
    f.r = J.r;
    f.M = J.M;
    f.n_cols = G.n_cols;
    f.refresh = J.sync == 0 ? 1 : 0;
    f.col = sr.col;
    f.box = box;
    f.vox_J = vox;
    f.xg_stride = xg_size(box.x1 - box.x0, box.y1 - box.y0, box.z1 - box.z0);
    f.n_groups = sr.n_groups;
    f.xg = J.xg;
    f.x = J.x;
    f.nx = G.nx;
    f.ny = G.ny;
    fin_body(G, f, L);
}

// Epoch-synchronous residual refresh over the epoch's touched row blocks
// (launched once per epoch, with c = 0).
__global__ __launch_bounds__(256) void kb_residual(BatchArgs B) {
    const int k = batch_job(B, blockIdx.x);
    const int L = blockIdx.x - B.prefix[k];
    const BJob J = cld(B.jobs, k);
    if (J.sync != 1) return;
    const int e = cld(B.ep, k);
    if (e < 0 || e >= J.n_epochs) return;
    const EpochRec er = cld(J.epochs, e);
    if (L * 4 >= er.uni_chunks) return;
    const DGeom G = J.G;
    ResArgs a{};
    a.ent = J.uni + er.uni_off;
    a.n_ent = er.n_uni;
    a.z = J.z;
    a.y = J.y;
    a.r = J.r;
    a.M = J.M;
    a.n_cols = G.n_cols;
    res_body(G, a, L, er.uni_chunks);
}

// End of a batch epoch: every job that had an epoch left moves to the next.
__global__ void kb_advance(BatchArgs B) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B.n_jobs) return;
    const int e = B.ep[k];
    if (e >= 0 && e < B.jobs[k].n_epochs) B.ep[k] = e + 1;
}

// ----------------------------------------------------------------------------
// utilities
// ----------------------------------------------------------------------------
__global__ void k_fill(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Partial sums of (y - p)^2 and y^2 per work-group (float64).
__global__ __launch_bounds__(256) void k_resnorm(const float* y, const float* p, int64_t n,
                                                 double* part) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double yy = y[i], d = yy - (double)p[i];
        a = fma(d, d, a);
        b = fma(yy, yy, b);
    }
    const double ta = block_sum256(a, sh);
    __syncthreads();
    const double tb = block_sum256(b, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

// Fixed-order sum of nblk (a, b) partial pairs into out[0], out[1] (one work-group).
__global__ __launch_bounds__(256) void k_sum_pairs(const double* part, int nblk, double* out) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    const double ta = block_sum256(a, sh);
    __syncthreads();
    const double tb = block_sum256(b, sh);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

// ----------------------------------------------------------------------------
// host-side launchers (internal linkage for the API file)
// ----------------------------------------------------------------------------
template <int MODE, int KS = kSplit>
static hipError_t launch_fwd_mode(const DGeom& G, const FwdArgs& a, hipStream_t st) {
    dim3 grid(a.n_chunks), block(MODE == 2 ? kChunk : kChunk * KS);
    const FwdCore c = a;
    switch (G.kind) {
        case kPar2D: hipLaunchKernelGGL((k_fwd<kPar2D, MODE, KS>), grid, block, 0, st, G, c); break;
        case kFanFlat: hipLaunchKernelGGL((k_fwd<kFanFlat, MODE, KS>), grid, block, 0, st, G, c); break;
        case kFanCurved: hipLaunchKernelGGL((k_fwd<kFanCurved, MODE, KS>), grid, block, 0, st, G, c); break;
        default: hipLaunchKernelGGL((k_fwd<kCone, MODE, KS>), grid, block, 0, st, G, c); break;
    }
    return hipGetLastError();
}

static hipError_t launch_fwd_inline(const DGeom& G, const FwdArgs& a, hipStream_t st) {
    dim3 grid(a.n_chunks), block(kChunk * kSplit);
    switch (G.kind) {
        case kPar2D: hipLaunchKernelGGL(k_fwd_inl<kPar2D>, grid, block, 0, st, G, a); break;
        case kFanFlat: hipLaunchKernelGGL(k_fwd_inl<kFanFlat>, grid, block, 0, st, G, a); break;
        case kFanCurved: hipLaunchKernelGGL(k_fwd_inl<kFanCurved>, grid, block, 0, st, G, a); break;
        default: hipLaunchKernelGGL(k_fwd_inl<kCone>, grid, block, 0, st, G, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_fwd(const DGeom& G, const FwdArgs& a, hipStream_t st) {
    if (a.n_chunks <= 0) return hipSuccess;
    if (!a.ent) {
        if (a.mode != 0) return hipErrorInvalidValue;     // inline entries: single mode only
        return launch_fwd_inline(G, a, st);
    }
    if (a.mode == 0) return launch_fwd_mode<0>(G, a, st);
    if (a.mode == 1) {
        // pieces per chord: a tuning choice of the fused step
        if (a.split == 1) return launch_fwd_mode<1, 1>(G, a, st);
        if (a.split == 2) return launch_fwd_mode<1, 2>(G, a, st);
        if (a.split == 4) return launch_fwd_mode<1, 4>(G, a, st);
        return hipErrorInvalidValue;
    }
    return launch_fwd_mode<2>(G, a, st);
}

template <class BA, int NW>
static void launch_back2(const DGeom& G, const BA& a, dim3 grid, hipStream_t st) {
    const dim3 block(64 * NW);
    switch (G.kind) {
        case kPar2D: hipLaunchKernelGGL((k_back2<kPar2D, BA, NW>), grid, block, 0, st, G, a); break;
        case kFanFlat: hipLaunchKernelGGL((k_back2<kFanFlat, BA, NW>), grid, block, 0, st, G, a); break;
        default: hipLaunchKernelGGL((k_back2<kFanCurved, BA, NW>), grid, block, 0, st, G, a); break;
    }
}

template <class BA>
static hipError_t launch_back_as(const DGeom& G, const BA& a, int n_groups, int waves, hipStream_t st) {
    const int nt = a.tiles_x * a.tiles_y * a.tiles_z;
    if (nt <= 0 || n_groups <= 0) return hipSuccess;
    const dim3 grid(nt, n_groups);
    if (G.kind == kCone && G.vertical) {
        hipLaunchKernelGGL(k_back3c<BA>, grid, dim3(256), 0, st, G, a);
    } else if (G.kind == kCone) {
        hipLaunchKernelGGL(k_back3<BA>, grid, dim3(256), 0, st, G, a);
    } else if (waves == 1) {
        launch_back2<BA, 1>(G, a, grid, st);
    } else if (waves == 2) {
        launch_back2<BA, 2>(G, a, grid, st);
    } else if (waves == 4) {
        launch_back2<BA, 4>(G, a, grid, st);
    } else if (waves == 8) {
        launch_back2<BA, 8>(G, a, grid, st);
    } else if (waves == 16) {
        launch_back2<BA, 16>(G, a, grid, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_back(const DGeom& G, const BackArgs& a, int n_groups, int waves, hipStream_t st) {
    if (!a.ent) return launch_back_as<BackArgs>(G, a, n_groups, waves, st);
    const BackCore c = a;
    return launch_back_as<BackCore>(G, c, n_groups, waves, st);
}

hipError_t launch_step(const StepArgs& s, int n_groups, hipStream_t st) {
    if (n_groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step, dim3(n_groups), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_finalize(const DGeom& G, const FinArgs& f, int vox_blocks, hipStream_t st) {
    const int nb = (f.n_chunks + 3) / 4 + vox_blocks;
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(256), 0, st, G, f);
    return hipGetLastError();
}

hipError_t launch_residual(const DGeom& G, const ResArgs& a, int n_chunks, hipStream_t st) {
    if (n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual, dim3((n_chunks + 3) / 4), dim3(256), 0, st, G, a, n_chunks);
    return hipGetLastError();
}

template <int KIND>
static hipError_t launch_batch_kind(int phase, const BatchArgs& b, int blocks, const Tune& t,
                                    hipStream_t st) {
    const dim3 grid(blocks);
    if (phase == kPhBack) {
        if constexpr (KIND == kCone || KIND == kConeV) {
            hipLaunchKernelGGL((kb_back<KIND, 4>), grid, dim3(256), 0, st, b);
        } else {
            if (t.waves == 1) hipLaunchKernelGGL((kb_back<KIND, 1>), grid, dim3(64), 0, st, b);
            else if (t.waves == 2) hipLaunchKernelGGL((kb_back<KIND, 2>), grid, dim3(128), 0, st, b);
            else if (t.waves == 4) hipLaunchKernelGGL((kb_back<KIND, 4>), grid, dim3(256), 0, st, b);
            else if (t.waves == 8) hipLaunchKernelGGL((kb_back<KIND, 8>), grid, dim3(512), 0, st, b);
            else if (t.waves == 16) hipLaunchKernelGGL((kb_back<KIND, 16>), grid, dim3(1024), 0, st, b);
            else return hipErrorInvalidValue;
        }
    } else {
        // the forward walk of a kConeV geometry is the cone's
        constexpr int FK = KIND == kConeV ? kCone : KIND;
        if (t.split == 1) hipLaunchKernelGGL((kb_fwd<FK, 1>), grid, dim3(kChunk), 0, st, b);
        else if (t.split == 2) hipLaunchKernelGGL((kb_fwd<FK, 2>), grid, dim3(2 * kChunk), 0, st, b);
        else if (t.split == 4) hipLaunchKernelGGL((kb_fwd<FK, 4>), grid, dim3(4 * kChunk), 0, st, b);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(int phase, int kind, const BatchArgs& b, int blocks, const Tune& t, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    switch (phase) {
        case kPhBack:
        case kPhFwd:
            switch (kind) {
                case kPar2D: return launch_batch_kind<kPar2D>(phase, b, blocks, t, st);
                case kFanFlat: return launch_batch_kind<kFanFlat>(phase, b, blocks, t, st);
                case kFanCurved: return launch_batch_kind<kFanCurved>(phase, b, blocks, t, st);
                case kConeV: return launch_batch_kind<kConeV>(phase, b, blocks, t, st);
                default: return launch_batch_kind<kCone>(phase, b, blocks, t, st);
            }
        case kPhStep: hipLaunchKernelGGL(kb_step, dim3(blocks), dim3(256), 0, st, b); break;
        case kPhFin: hipLaunchKernelGGL(kb_finalize, dim3(blocks), dim3(256), 0, st, b); break;
        default: hipLaunchKernelGGL(kb_residual, dim3(blocks), dim3(256), 0, st, b); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchArgs& b, hipStream_t st) {
    if (b.n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_advance, dim3((b.n_jobs + 255) / 256), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_resnorm(const float* y, const float* p, int64_t n, double* part, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_resnorm, dim3(nblk), dim3(256), 0, st, y, p, n, part);
    return hipGetLastError();
}

hipError_t launch_sum_pairs(const double* part, int nblk, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, st, part, nblk, out);
    return hipGetLastError();
}

}  // namespace ct
