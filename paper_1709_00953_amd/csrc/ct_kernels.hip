// gfx950 kernels of the block-iterative CT solver.
//
//  k_fwd      ray-driven Siddon forward projection A_I^J x_J through one
//             column block (Alg. 3 last line; Eq. 12-13).  One lane per ray,
//             consecutive lanes = consecutive detector bins, so the output
//             writes are coalesced along the detector-major ray layout.  The
//             ray is set up in float64 (entry into the box), then walked in
//             float32 box-local voxel coordinates, crossing parameters taken
//             from the plane index rather than by repeated addition.  The
//             fused mode walks x_J and g_J together (A x and A g in one pass)
//             and emits a float64 partial of ||A g||^2 per work-group; the
//             count mode counts the pairs longer than tau (block densities).
//  k_back2/3  gather back-projection (A_I^J)^T r_I (Eq. 7): one lane per
//             voxel, which visits the bins of its shadow in every view of the
//             group and clips each candidate ray against its own box, so no
//             two lanes write the same output and no atomics are needed.
//             The voxel's view-frame offset and each candidate's distance from
//             the voxel centre are formed in float64 (they cancel ~500 mm
//             lever arms); the clip itself is float32.
//  k_step     mu = beta ||g||^2 / ||A g||^2 per group (Eq. 11, relaxed), from
//             fixed-order float64 sums of the per-work-group partials.
//  k_finalize z^J_{I_G} = A x + mu A g, residual r = y - sum_j z^j on the
//             touched rays (Sec. II-C), and x_J = mean_G (x_J + mu_G g_G).
//  k_residual r_I = y_I - sum_j z^j_I (epoch-synchronous refresh, reset).
//
// No work-group ever writes an address another one writes (except integer
// atomics of the density count), so every result is reproducible bit for bit.
#include "ct_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

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

template <class A>
__device__ __forceinline__ Entry get_entry(const A& a, int i) {
    return a.ent ? a.ent[i] : a.inl[i];
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
        const Ray2& R = G.ray2[(size_t)view * G.nu + iu];
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
template <int KIND, int MODE>
__global__ __launch_bounds__(256) void k_fwd(DGeom G, FwdArgs a) {
    constexpr int DIMS = (KIND == kCone) ? 3 : 2;
    constexpr bool DIVERGENT = (KIND != kPar2D);
    __shared__ double sh[4];
    __shared__ unsigned shu[4];

    const int bid = blockIdx.x;
    const int ei = find_entry(a, bid);
    const Entry en = get_entry(a, ei);
    const int rb = en.rb;
    const Chunk ch = G.chunks[G.rb_chunk_ptr[rb] + (bid - en.chunk_prefix)];
    const Tile tl = G.tiles[ch.tile];
    const int lane = threadIdx.x;
    const bool active = lane < ch.cnt;

    float acc = 0.f, acc2 = 0.f;
    unsigned cnt = 0;
    int ray = 0;
    if (active) {
        const int w = tl.u1 - tl.u0;
        const int k = ch.k0 + lane;
        const int iv = tl.v0 + k / w;
        const int iu = tl.u0 + k % w;
        ray = (tl.view * G.nv + iv) * G.nu + iu;

        double o[3], d[3];
        ray_of<KIND>(G, tl.view, iv, iu, o, d);
        const double h[3] = {G.vx, G.vy, G.vz};
        const double org[3] = {G.ox, G.oy, G.oz};
        const int b0[3] = {a.box.x0, a.box.y0, a.box.z0};
        const int b1[3] = {a.box.x1, a.box.y1, a.box.z1};
        double t0 = DIVERGENT ? 0.0 : -INFINITY, t1 = INFINITY;
        bool hit = true;
        double lo[3];
#pragma unroll
        for (int k2 = 0; k2 < DIMS; ++k2) {
            lo[k2] = fma((double)b0[k2], h[k2], org[k2]);
            const double hi = fma((double)b1[k2], h[k2], org[k2]);
            if (d[k2] == 0.0) {
                hit = hit && (o[k2] >= lo[k2]) && (o[k2] < hi);
            } else {
                const double inv = 1.0 / d[k2];
                const double ta = (lo[k2] - o[k2]) * inv;
                const double tb = (hi - o[k2]) * inv;
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
        }
        hit = hit && (t1 > t0);
        if (hit) {
            // box-local entry point in voxel units and per-axis stepping
            int nb[3], ii[3], sg[3];
            float dl[3], inv[3], tk[3];
            int stride[3];
            const int nxJ = a.box.x1 - a.box.x0, nyJ = a.box.y1 - a.box.y0;
            if constexpr (MODE == 1) {
                stride[0] = 1;
                stride[1] = nxJ;
                stride[2] = nxJ * nyJ;
            } else {
                stride[0] = 1;
                stride[1] = G.nx;
                stride[2] = G.nx * G.ny;
            }
            const float T = (float)(t1 - t0);
#pragma unroll
            for (int k2 = 0; k2 < DIMS; ++k2) {
                nb[k2] = b1[k2] - b0[k2];
                const double e = (fma(t0, d[k2], o[k2]) - lo[k2]) / h[k2];
                const float ef = (float)e;
                int i = (int)floorf(ef);
                if (d[k2] < 0.0 && (float)i == ef) i -= 1;
                i = min(max(i, 0), nb[k2] - 1);
                ii[k2] = i;
                if (d[k2] > 0.0) {
                    sg[k2] = 1;
                    dl[k2] = (float)(i + 1) - ef;
                    inv[k2] = (float)(h[k2] / d[k2]);
                    tk[k2] = dl[k2] * inv[k2];
                } else if (d[k2] < 0.0) {
                    sg[k2] = -1;
                    dl[k2] = ef - (float)i;
                    inv[k2] = (float)(-h[k2] / d[k2]);
                    tk[k2] = dl[k2] * inv[k2];
                } else {
                    sg[k2] = 0;
                    dl[k2] = 0.f;
                    inv[k2] = 0.f;
                    tk[k2] = INFINITY;
                }
            }
            int idx;
            if constexpr (MODE == 1) {
                idx = ii[0] + ii[1] * stride[1] + (DIMS == 3 ? ii[2] * stride[2] : 0);
            } else {
                idx = (a.box.x0 + ii[0]) + (a.box.y0 + ii[1]) * stride[1] +
                      (DIMS == 3 ? (a.box.z0 + ii[2]) * stride[2] : 0);
            }
            const float2* xg = (MODE == 1) ? a.xg + (size_t)en.group * a.vox_J : nullptr;
            const int maxit = nb[0] + nb[1] + (DIMS == 3 ? nb[2] : 0) + 4;
            float tau = 0.f;
            for (int it = 0; it < maxit; ++it) {
                float tn = fminf(tk[0], tk[1]);
                if constexpr (DIMS == 3) tn = fminf(tn, tk[2]);
                tn = fminf(tn, T);
                const float len = tn - tau;
                if constexpr (MODE == 0) {
                    acc = fmaf(len, a.x[idx], acc);
                } else if constexpr (MODE == 1) {
                    const float2 v = xg[idx];
                    acc = fmaf(len, v.x, acc);
                    acc2 = fmaf(len, v.y, acc2);
                } else {
                    cnt += (len > a.tau) ? 1u : 0u;
                }
                if (tn >= T) break;
                tau = tn;
                int ax;
                if constexpr (DIMS == 3) {
                    ax = (tk[0] <= tk[1]) ? ((tk[0] <= tk[2]) ? 0 : 2) : ((tk[1] <= tk[2]) ? 1 : 2);
                } else {
                    ax = (tk[0] <= tk[1]) ? 0 : 1;
                }
                // branch-free advance of axis `ax`
                bool out = false;
#pragma unroll
                for (int k2 = 0; k2 < DIMS; ++k2) {
                    if (ax == k2) {
                        ii[k2] += sg[k2];
                        idx += sg[k2] * stride[k2];
                        dl[k2] += 1.f;
                        tk[k2] = dl[k2] * inv[k2];
                        out = (unsigned)ii[k2] >= (unsigned)nb[k2];
                    }
                }
                if (out) break;
            }
        }
    }

    if constexpr (MODE == 0) {
        if (active) a.out[ray] = (a.flags & 1) ? a.out[ray] + acc : acc;
    } else if constexpr (MODE == 1) {
        if (active) {
            a.out[ray] = acc;
            a.q[en.slot_prefix + ch.roff + lane] = acc2;
        }
        const double p = active ? (double)acc2 * (double)acc2 : 0.0;
        const double t = block_sum256(p, sh);
        if (threadIdx.x == 0) a.partial[bid] = t;
    } else {
        unsigned c = wave_sum_u(cnt);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) shu[w] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = (unsigned long long)shu[0] + shu[1] + shu[2] + shu[3];
            if (tot) atomicAdd(a.nnz + (size_t)rb * a.n_cols + a.col, tot);
        }
    }
}

// ----------------------------------------------------------------------------
// K1: gather back-projection, 2D
// ----------------------------------------------------------------------------
// Clip length of the ray described by R with the voxel whose centre lies at
// signed distance delta from it.
__device__ __forceinline__ float chord2(float delta, const Ray2& R) {
    const float cx = delta * R.kx, cy = delta * R.ky;
    const float hi = fminf(cx + R.wx, cy + R.wy);
    const float lo = fmaxf(cx - R.wx, cy - R.wy);
    return fmaxf(hi - lo, 0.f);
}

// Same, for rays with an exactly zero direction component (half-open voxels).
__device__ __forceinline__ float chord2_axis(float delta, const Ray2& R, float hx, float hy) {
    if (R.wx < 0.f) {
        const float off = delta * R.kx;
        return (off >= -hx && off < hx) ? 2.f * R.wy : 0.f;
    }
    if (R.wy < 0.f) {
        const float off = delta * R.ky;
        return (off >= -hy && off < hy) ? 2.f * R.wx : 0.f;
    }
    return chord2(delta, R);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_back2(DGeom G, BackArgs a) {
    __shared__ double sh[4];
    const int gi = blockIdx.y;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int lx = threadIdx.x & (kTile2 - 1), ly = threadIdx.x / kTile2;
    const int ix = a.box.x0 + tx * kTile2 + lx, iy = a.box.y0 + ty * kTile2 + ly;
    const bool valid = ix < a.box.x1 && iy < a.box.y1;

    const double cx = G.ox + ((double)ix + 0.5) * G.vx;
    const double cy = G.oy + ((double)iy + 0.5) * G.vy;
    const float hx = (float)(0.5 * G.vx), hy = (float)(0.5 * G.vy);
    const float R = G.radius;
    const float c0 = 0.5f * (float)(G.nu - 1);
    const float ipu = (float)(1.0 / G.pu);
    float acc = 0.f;

    int e0 = 0, e1 = a.n_ent;
    if (a.gptr) {
        e0 = a.gptr[gi];
        e1 = a.gptr[gi + 1];
    }
    if (valid) {
        for (int e = e0; e < e1; ++e) {
            const int rb = get_entry(a, e).rb;
            const int t_end = G.rb_tile_ptr[rb + 1];
            for (int t = G.rb_tile_ptr[rb]; t < t_end; ++t) {
                const Tile tl = G.tiles[t];
                const int view = tl.view;
                const double* V = view_of(G, view);
                double A, B;
                float beta, wb;
                if constexpr (KIND == kPar2D) {
                    // signed distance of the bin-u ray: delta = B - u*kappa
                    A = 1.0;
                    B = V[0] * (cy - V[4]) - V[1] * (cx - V[3]);
                    const float kap = (float)V[15];
                    beta = (float)(B / V[15]) * ipu + c0;
                    wb = R / fabsf(kap) * ipu;
                } else {
                    const double qx = cx - V[0], qy = cy - V[1];
                    A = fma(qx, V[12], qy * V[13]);
                    B = fma(qx, V[6], qy * V[7]);
                    const float Af = (float)A, Bf = (float)B;
                    if constexpr (KIND == kFanCurved) {
                        const float phi = atan2f(Bf, Af);
                        const float rho2 = fmaf(Af, Af, Bf * Bf);
                        beta = phi * ipu + c0;
                        wb = R * rsqrtf(fmaxf(rho2 - R * R, 1e-30f)) * ipu;
                    } else {
                        const float sdd = (float)V[15];
                        const float t = Bf / Af;
                        beta = sdd * t * ipu + c0;
                        wb = sdd * R * (1.f + fabsf(t)) / (Af - R) * ipu;
                    }
                }
                int blo = (int)ceilf(beta - wb - 1e-3f);
                int bhi = (int)floorf(beta + wb + 1e-3f);
                blo = max(blo, tl.u0);
                bhi = min(bhi, tl.u1 - 1);
                const Ray2* RR = G.ray2 + (size_t)view * G.nu;
                const float* rr = a.r + (size_t)view * G.nu;
                if (G.view_flags[view] & 1) {
                    for (int b = blo; b <= bhi; ++b) {
                        const Ray2 Rb = RR[b];
                        const float dlt = (float)fma(Rb.p, B, -Rb.q * A);
                        acc = fmaf(chord2_axis(dlt, Rb, hx, hy), rr[b], acc);
                    }
                } else {
                    for (int b = blo; b <= bhi; ++b) {
                        const Ray2 Rb = RR[b];
                        const float dlt = (float)fma(Rb.p, B, -Rb.q * A);
                        acc = fmaf(chord2(dlt, Rb), rr[b], acc);
                    }
                }
            }
        }
    }

    const int nxJ = a.box.x1 - a.box.x0;
    if (a.fused) {
        if (valid) {
            const int li = (iy - a.box.y0) * nxJ + (ix - a.box.x0);
            const int gix = iy * G.nx + ix;
            a.xg[(size_t)gi * a.vox_J + li] = make_float2(a.x[gix], acc);
        }
        const double p = valid ? (double)acc * (double)acc : 0.0;
        const double t = block_sum256(p, sh);
        if (threadIdx.x == 0) a.partial[(size_t)gi * gridDim.x + blockIdx.x] = t;
    } else if (valid) {
        const int gix = iy * G.nx + ix;
        a.g[gix] = (a.flags & 1) ? a.g[gix] + acc : acc;
    }
}

// ----------------------------------------------------------------------------
// K1: gather back-projection, 3D cone
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_back3(DGeom G, BackArgs a) {
    __shared__ double sh[4];
    const int gi = blockIdx.y;
    const int bt = blockIdx.x;
    const int tx = bt % a.tiles_x;
    const int ty = (bt / a.tiles_x) % a.tiles_y;
    const int tz = bt / (a.tiles_x * a.tiles_y);
    const int lx = threadIdx.x & 7, ly = (threadIdx.x >> 3) & 7, lz = threadIdx.x >> 6;
    const int ix = a.box.x0 + tx * kTile3x + lx;
    const int iy = a.box.y0 + ty * kTile3y + ly;
    const int iz = a.box.z0 + tz * kTile3z + lz;
    const bool valid = ix < a.box.x1 && iy < a.box.y1 && iz < a.box.z1;

    const double c[3] = {G.ox + ((double)ix + 0.5) * G.vx, G.oy + ((double)iy + 0.5) * G.vy,
                         G.oz + ((double)iz + 0.5) * G.vz};
    const float hh[3] = {(float)(0.5 * G.vx), (float)(0.5 * G.vy), (float)(0.5 * G.vz)};
    const float R = G.radius;
    const float c0u = 0.5f * (float)(G.nu - 1), c0v = 0.5f * (float)(G.nv - 1);
    const float ipu = (float)(1.0 / G.pu), ipv = (float)(1.0 / G.pv);
    float acc = 0.f;

    int e0 = 0, e1 = a.n_ent;
    if (a.gptr) {
        e0 = a.gptr[gi];
        e1 = a.gptr[gi + 1];
    }
    if (valid) {
        for (int e = e0; e < e1; ++e) {
            const int rb = get_entry(a, e).rb;
            const int t_end = G.rb_tile_ptr[rb + 1];
            for (int t = G.rb_tile_ptr[rb]; t < t_end; ++t) {
                const Tile tl = G.tiles[t];
                const int view = tl.view;
                const double* V = view_of(G, view);
                const double q[3] = {c[0] - V[0], c[1] - V[1], c[2] - V[2]};
                const double A = fma(q[0], V[12], fma(q[1], V[13], q[2] * V[14]));
                const double Bu = fma(q[0], V[6], fma(q[1], V[7], q[2] * V[8]));
                const double Bv = fma(q[0], V[9], fma(q[1], V[10], q[2] * V[11]));
                const double sdd = V[15];
                const double tc = A * V[16];            // ray parameter at the voxel's depth
                const float Af = (float)A;
                const float tu = (float)Bu / Af, tv = (float)Bv / Af;
                const float sd = (float)sdd;
                const float den = sd * R / (Af - R);
                const float betu = sd * tu * ipu + c0u, betv = sd * tv * ipv + c0v;
                const float wu = den * (1.f + fabsf(tu)) * ipu, wv = den * (1.f + fabsf(tv)) * ipv;
                const int ulo = max((int)ceilf(betu - wu - 1e-3f), tl.u0);
                const int uhi = min((int)floorf(betu + wu + 1e-3f), tl.u1 - 1);
                const int vlo = max((int)ceilf(betv - wv - 1e-3f), tl.v0);
                const int vhi = min((int)floorf(betv + wv + 1e-3f), tl.v1 - 1);
                const bool careful = (G.view_flags[view] & 1) != 0;
                for (int iv = vlo; iv <= vhi; ++iv) {
                    const double v = ((double)iv - 0.5 * (double)(G.nv - 1)) * G.pv;
                    const float* rr = a.r + ((size_t)view * G.nv + iv) * G.nu;
                    for (int iu = ulo; iu <= uhi; ++iu) {
                        const double u = ((double)iu - 0.5 * (double)(G.nu - 1)) * G.pu;
                        const double D[3] = {fma(v, V[9], fma(u, V[6], sdd * V[12])),
                                             fma(v, V[10], fma(u, V[7], sdd * V[13])),
                                             fma(v, V[11], fma(u, V[8], sdd * V[14]))};
                        float lo = -INFINITY, hi = INFINITY;
                        bool member = true;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            const float w = (float)fma(-tc, D[k], q[k]);
                            const float Dk = (float)D[k];
                            if (careful && Dk == 0.f) {
                                member = member && (w > -hh[k]) && (w <= hh[k]);
                            } else {
                                const float inv = 1.f / Dk;
                                const float ta = (w - hh[k]) * inv, tb = (w + hh[k]) * inv;
                                lo = fmaxf(lo, fminf(ta, tb));
                                hi = fminf(hi, fmaxf(ta, tb));
                            }
                        }
                        const float Df0 = (float)D[0], Df1 = (float)D[1], Df2 = (float)D[2];
                        const float nrm = sqrtf(fmaf(Df0, Df0, fmaf(Df1, Df1, Df2 * Df2)));
                        const float L = member ? fmaxf(hi - lo, 0.f) * nrm : 0.f;
                        acc = fmaf(L, rr[iu], acc);
                    }
                }
            }
        }
    }

    const int nxJ = a.box.x1 - a.box.x0, nyJ = a.box.y1 - a.box.y0;
    const size_t gix = ((size_t)iz * G.ny + iy) * G.nx + ix;
    if (a.fused) {
        if (valid) {
            const int li = ((iz - a.box.z0) * nyJ + (iy - a.box.y0)) * nxJ + (ix - a.box.x0);
            a.xg[(size_t)gi * a.vox_J + li] = make_float2(a.x[gix], acc);
        }
        const double p = valid ? (double)acc * (double)acc : 0.0;
        const double t = block_sum256(p, sh);
        if (threadIdx.x == 0) a.partial[(size_t)gi * gridDim.x + blockIdx.x] = t;
    } else if (valid) {
        a.g[gix] = (a.flags & 1) ? a.g[gix] + acc : acc;
    }
}

// ----------------------------------------------------------------------------
// K3: step sizes
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_step(StepArgs s) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    const int c0 = s.ent[s.gptr[g]].chunk_prefix;
    const int e_next = s.gptr[g + 1];
    const int c1 = (e_next < s.gptr[gridDim.x]) ? s.ent[e_next].chunk_prefix : s.n_chunks;
    double gg = 0.0, qq = 0.0;
    for (int t = lane; t < s.n_tiles; t += 64) gg += s.pg[(size_t)g * s.n_tiles + t];
    for (int c = c0 + lane; c < c1; c += 64) qq += s.pq[c];
    gg = wave_sum(gg);
    qq = wave_sum(qq);
    if (lane == 0) s.mu[g] = (gg > 0.0 && qq > 0.0) ? s.beta[g] * gg / qq : 0.0;
}

// ----------------------------------------------------------------------------
// K4: finalize a column-block step
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_finalize(DGeom G, FinArgs f) {
    const int bid = blockIdx.x;
    if (bid < f.n_chunks) {
        const int ei = find_entry(f, bid);
        const Entry en = get_entry(f, ei);
        const Chunk ch = G.chunks[G.rb_chunk_ptr[en.rb] + (bid - en.chunk_prefix)];
        const int lane = threadIdx.x;
        if (lane >= ch.cnt) return;
        const Tile tl = G.tiles[ch.tile];
        const int w = tl.u1 - tl.u0;
        const int k = ch.k0 + lane;
        const int ray = (tl.view * G.nv + tl.v0 + k / w) * G.nu + tl.u0 + k % w;
        const float mu = (float)f.mu[en.group];
        const float zn = fmaf(mu, f.q[en.slot_prefix + ch.roff + lane], f.zJ[ray]);
        f.zJ[ray] = zn;
        if (f.refresh) {
            float s = 0.f;
            for (int j = 0; j < f.n_cols; ++j) s += f.z[(size_t)j * f.M + ray];
            f.r[ray] = f.y[ray] - s;
        }
    } else {
        const int v = (bid - f.n_chunks) * 256 + threadIdx.x;
        if (v >= f.vox_J) return;
        float s = 0.f;
        for (int g = 0; g < f.n_groups; ++g) {
            const float2 p = f.xg[(size_t)g * f.vox_J + v];
            s += fmaf((float)f.mu[g], p.y, p.x);
        }
        const int nxJ = f.box.x1 - f.box.x0, nyJ = f.box.y1 - f.box.y0;
        const int lx = v % nxJ, ly = (v / nxJ) % nyJ, lz = v / (nxJ * nyJ);
        const size_t gix = ((size_t)(f.box.z0 + lz) * f.ny + (f.box.y0 + ly)) * f.nx + f.box.x0 + lx;
        f.x[gix] = s / (float)f.n_groups;
    }
}

// ----------------------------------------------------------------------------
// K5: residual refresh over the rays of a list of row blocks
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_residual(DGeom G, ResArgs a) {
    const int bid = blockIdx.x;
    const int ei = find_entry(a, bid);
    const Entry en = get_entry(a, ei);
    const Chunk ch = G.chunks[G.rb_chunk_ptr[en.rb] + (bid - en.chunk_prefix)];
    const int lane = threadIdx.x;
    if (lane >= ch.cnt) return;
    const Tile tl = G.tiles[ch.tile];
    const int w = tl.u1 - tl.u0;
    const int k = ch.k0 + lane;
    const int ray = (tl.view * G.nv + tl.v0 + k / w) * G.nu + tl.u0 + k % w;
    float s = 0.f;
    for (int j = 0; j < a.n_cols; ++j) s += a.z[(size_t)j * a.M + ray];
    a.r[ray] = a.y[ray] - s;
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

// ----------------------------------------------------------------------------
// host-side launchers (internal linkage for the API file)
// ----------------------------------------------------------------------------
template <int MODE>
static hipError_t launch_fwd_mode(const DGeom& G, const FwdArgs& a, hipStream_t st) {
    dim3 grid(a.n_chunks), block(256);
    switch (G.kind) {
        case kPar2D: hipLaunchKernelGGL((k_fwd<kPar2D, MODE>), grid, block, 0, st, G, a); break;
        case kFanFlat: hipLaunchKernelGGL((k_fwd<kFanFlat, MODE>), grid, block, 0, st, G, a); break;
        case kFanCurved: hipLaunchKernelGGL((k_fwd<kFanCurved, MODE>), grid, block, 0, st, G, a); break;
        default: hipLaunchKernelGGL((k_fwd<kCone, MODE>), grid, block, 0, st, G, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_fwd(const DGeom& G, const FwdArgs& a, hipStream_t st) {
    if (a.n_chunks <= 0) return hipSuccess;
    if (a.mode == 0) return launch_fwd_mode<0>(G, a, st);
    if (a.mode == 1) return launch_fwd_mode<1>(G, a, st);
    return launch_fwd_mode<2>(G, a, st);
}

hipError_t launch_back(const DGeom& G, const BackArgs& a, int n_groups, hipStream_t st) {
    const int nt = a.tiles_x * a.tiles_y * a.tiles_z;
    if (nt <= 0 || n_groups <= 0) return hipSuccess;
    dim3 grid(nt, n_groups), block(256);
    switch (G.kind) {
        case kPar2D: hipLaunchKernelGGL(k_back2<kPar2D>, grid, block, 0, st, G, a); break;
        case kFanFlat: hipLaunchKernelGGL(k_back2<kFanFlat>, grid, block, 0, st, G, a); break;
        case kFanCurved: hipLaunchKernelGGL(k_back2<kFanCurved>, grid, block, 0, st, G, a); break;
        default: hipLaunchKernelGGL(k_back3, grid, block, 0, st, G, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs& s, int n_groups, hipStream_t st) {
    if (n_groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step, dim3(n_groups), dim3(64), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_finalize(const DGeom& G, const FinArgs& f, int vox_blocks, hipStream_t st) {
    const int nb = f.n_chunks + vox_blocks;
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(256), 0, st, G, f);
    return hipGetLastError();
}

hipError_t launch_residual(const DGeom& G, const ResArgs& a, int n_chunks, hipStream_t st) {
    if (n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual, dim3(n_chunks), dim3(256), 0, st, G, a);
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

}  // namespace ct
