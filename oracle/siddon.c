/*
 * FP64 Siddon row generator for the oracle (test infrastructure only).
 *
 * System matrix of Sec. II-A: A_ij is the intersection length (mm) of ray i
 * with voxel j, computed by a Siddon traversal (the paper cites the fast
 * Siddon variant of Jacobs et al.):
 *   1. clip the line to the volume box (slab method); a divergent ray starts
 *      at its source (t >= 0);
 *   2. collect every grid-plane crossing strictly inside the clipped range,
 *      sort them, and cut the range into segments;
 *   3. each segment of positive length belongs to the voxel that contains its
 *      midpoint (half-open voxels; reading C12), its length is (t1-t0)*|d|;
 *   4. entries of the same voxel are merged and the row is sorted by column.
 * A direction component that is exactly zero yields no crossings on that
 * axis; such a ray is inside the volume slab iff lo <= o < hi.
 *
 * Plain, slow and obviously correct: no incremental stepping, one qsort per
 * row.  OpenMP over rays only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dims;              /* 2 or 3 */
    int n[3];              /* voxels per axis */
    double lo[3];          /* volume min corner */
    double h[3];           /* voxel pitch */
} vol_t;

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

typedef struct { int64_t j; double v; } ent_t;

static int cmp_ent(const void* a, const void* b) {
    int64_t x = ((const ent_t*)a)->j, y = ((const ent_t*)b)->j;
    return (x > y) - (x < y);
}

/* Clip parameter range of the line o + t d against the volume box. */
static int clip_volume(const vol_t* V, const double* o, const double* d, int divergent,
                       double* t0, double* t1) {
    double a = -INFINITY, b = INFINITY;
    if (divergent) a = 0.0;
    for (int k = 0; k < V->dims; ++k) {
        double lo = V->lo[k], hi = V->lo[k] + V->n[k] * V->h[k];
        if (d[k] == 0.0) {
            if (!(o[k] >= lo && o[k] < hi)) return 0;
            continue;
        }
        double ta = (lo - o[k]) / d[k], tb = (hi - o[k]) / d[k];
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > a) a = ta;
        if (tb < b) b = tb;
    }
    *t0 = a; *t1 = b;
    return b > a;
}

/* Fill one row into ent (capacity cap); returns number of entries. */
static int64_t row(const vol_t* V, const double* o, const double* d, int divergent,
                   double* tbuf, ent_t* ent) {
    double t0, t1;
    if (!clip_volume(V, o, d, divergent, &t0, &t1)) return 0;
    int64_t nt = 0;
    tbuf[nt++] = t0;
    for (int k = 0; k < V->dims; ++k) {
        if (d[k] == 0.0) continue;
        for (int p = 0; p <= V->n[k]; ++p) {
            double t = (V->lo[k] + p * V->h[k] - o[k]) / d[k];
            if (t > t0 && t < t1) tbuf[nt++] = t;
        }
    }
    tbuf[nt++] = t1;
    qsort(tbuf, (size_t)nt, sizeof(double), cmp_double);
    double dn = 0.0;
    for (int k = 0; k < V->dims; ++k) dn += d[k] * d[k];
    dn = sqrt(dn);
    int64_t ne = 0;
    for (int64_t q = 0; q + 1 < nt; ++q) {
        double len = (tbuf[q + 1] - tbuf[q]) * dn;
        if (!(len > 1e-12)) continue;
        double tm = 0.5 * (tbuf[q] + tbuf[q + 1]);
        int64_t idx[3] = {0, 0, 0};
        for (int k = 0; k < V->dims; ++k) {
            double c = (o[k] + tm * d[k] - V->lo[k]) / V->h[k];
            int64_t ic = (int64_t)floor(c);
            if (ic < 0) ic = 0;
            if (ic >= V->n[k]) ic = V->n[k] - 1;
            idx[k] = ic;
        }
        int64_t j = idx[0] + (int64_t)V->n[0] * (idx[1] + (int64_t)V->n[1] * idx[2]);
        ent[ne].j = j;
        ent[ne].v = len;
        ++ne;
    }
    if (ne > 1) {
        qsort(ent, (size_t)ne, sizeof(ent_t), cmp_ent);
        int64_t w = 0;
        for (int64_t q = 1; q < ne; ++q) {
            if (ent[q].j == ent[w].j) ent[w].v += ent[q].v;
            else ent[++w] = ent[q];
        }
        ne = w + 1;
    }
    return ne;
}

static void setup(vol_t* V, int dims, const int64_t* n, const double* lo, const double* h) {
    V->dims = dims;
    for (int k = 0; k < 3; ++k) {
        V->n[k] = (k < dims) ? (int)n[k] : 1;
        V->lo[k] = lo[k];
        V->h[k] = h[k];
    }
}

static int64_t cap_for(const vol_t* V) {
    int64_t c = 2;
    for (int k = 0; k < V->dims; ++k) c += V->n[k] + 1;
    return c;
}

/* Pass 1: number of entries per ray. */
int siddon_count(int dims, const int64_t* n, const double* lo, const double* h,
                 int64_t n_rays, const double* org, const double* dir, int divergent,
                 int64_t* counts) {
    vol_t V;
    setup(&V, dims, n, lo, h);
    int64_t cap = cap_for(&V);
    int err = 0;
#pragma omp parallel
    {
        double* tb = (double*)malloc(sizeof(double) * cap);
        ent_t* eb = (ent_t*)malloc(sizeof(ent_t) * cap);
        if (!tb || !eb) err = 1;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n_rays; ++i) {
            if (tb && eb) counts[i] = row(&V, org + 3 * i, dir + 3 * i, divergent, tb, eb);
        }
        free(tb);
        free(eb);
    }
    return err;
}

/* Pass 2: fill CSR arrays given row pointers from pass 1. */
int siddon_fill(int dims, const int64_t* n, const double* lo, const double* h,
                int64_t n_rays, const double* org, const double* dir, int divergent,
                const int64_t* indptr, int64_t* indices, double* data) {
    vol_t V;
    setup(&V, dims, n, lo, h);
    int64_t cap = cap_for(&V);
    int err = 0;
#pragma omp parallel
    {
        double* tb = (double*)malloc(sizeof(double) * cap);
        ent_t* eb = (ent_t*)malloc(sizeof(ent_t) * cap);
        if (!tb || !eb) err = 1;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n_rays; ++i) {
            if (!(tb && eb)) continue;
            int64_t ne = row(&V, org + 3 * i, dir + 3 * i, divergent, tb, eb);
            int64_t base = indptr[i];
            if (base + ne != indptr[i + 1]) { err = 2; continue; }
            for (int64_t q = 0; q < ne; ++q) {
                indices[base + q] = eb[q].j;
                data[base + q] = eb[q].v;
            }
        }
        free(tb);
        free(eb);
    }
    return err;
}

/* Thread count of the OpenMP ray loops above (a timing knob only: every ray
 * is computed the same way whatever the count). */
#include <omp.h>
void siddon_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int siddon_max_threads(void) { return omp_get_max_threads(); }
