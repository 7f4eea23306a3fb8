/*
 * spmvgen.c -- seeded synthetic sparse-matrix generators.
 *
 * Builds the CRS inputs (0-based IRP/ICOL/VAL, the arrays of the paper's
 * section 2.1) for the stencil, power-law, banded and row-length-sweep
 * workloads, and the dense vectors x.  This module holds no arithmetic of the
 * method itself: no transformation, no SpMV, no D_mat.  It is shared, as an
 * input source only, by the CPU oracle tests and by the GPU path.
 *
 * Randomness is counter based: every draw is a pure function of
 * (seed, stream, counter) through SplitMix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), so the
 * output does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* One 64-bit draw for counter `ctr` of stream `stream` under `seed`. */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    return sm64(sm64(seed ^ sm64(stream)) + ctr);
}

/* Uniform double in [0,1) with 53 random bits. */
static inline double unif(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    return (double)(draw(seed, stream, ctr) >> 11) * 0x1.0p-53;
}

/* Standard normal by Box-Muller from counters 2c and 2c+1. */
static inline double normal(uint64_t seed, uint64_t stream, uint64_t c)
{
    double u1 = unif(seed, stream, 2 * c);
    double u2 = unif(seed, stream, 2 * c + 1);
    return sqrt(-2.0 * log1p(-u1)) * cos(6.283185307179586476925 * u2);
}

/* Uniform integer in [0, m) (multiply-shift, bias < m / 2^64). */
static inline uint64_t below(uint64_t seed, uint64_t stream, uint64_t ctr, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)draw(seed, stream, ctr) * m) >> 64);
}

enum { ST_X = 1, ST_VAL = 2, ST_LEN = 3, ST_COL = 4, ST_MISC = 5 };

/* ---------------------------------------------------------------- vectors */

void gen_uniform(int64_t m, double lo, double hi, uint64_t seed, uint64_t stream, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        out[i] = lo + (hi - lo) * unif(seed, stream, (uint64_t)i);
}

void gen_normal(int64_t m, uint64_t seed, uint64_t stream, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        out[i] = normal(seed, stream, (uint64_t)i);
}

/* ------------------------------------------------------- 2-D 5-point grid */

/* Row i = x + nx*y couples to i-nx, i-1, i, i+1, i+nx inside the grid;
 * columns ascending.  Returns nnz; fills the arrays when they are non-NULL.
 * diag/off are the diagonal and off-diagonal values. */
int64_t gen_lap2d(int32_t nx, int32_t ny, double diag, double off,
                  int32_t *irp, int32_t *icol, double *val)
{
    int64_t p = 0;
    int32_t n = nx * ny;
    for (int32_t i = 0; i < n; ++i) {
        int32_t x = i % nx, y = i / nx;
        if (irp) irp[i] = (int32_t)p;
        int32_t cols[5];
        double vals[5];
        int c = 0;
        if (y > 0)      { cols[c] = i - nx; vals[c++] = off; }
        if (x > 0)      { cols[c] = i - 1;  vals[c++] = off; }
        cols[c] = i; vals[c++] = diag;
        if (x < nx - 1) { cols[c] = i + 1;  vals[c++] = off; }
        if (y < ny - 1) { cols[c] = i + nx; vals[c++] = off; }
        for (int k = 0; k < c; ++k, ++p) {
            if (icol) icol[p] = cols[k];
            if (val) val[p] = vals[k];
        }
    }
    if (irp) irp[n] = (int32_t)p;
    return p;
}

/* ------------------------------------------------ 3-D 27-point stencil */

static inline int32_t span3(int32_t c, int32_t m) { return (c > 0) + 1 + (c < m - 1); }

/* Row i = x + nx*(y + ny*z) couples to every (x+dx, y+dy, z+dz) with
 * dx,dy,dz in {-1,0,1} inside the box (Dirichlet truncation); columns
 * ascending.  Values: integer_values != 0 gives diagonal 26, neighbours -1;
 * otherwise diagonal 26 + U[0,1) and neighbours -1 + U[-0.1,0.1) drawn per
 * entry from (seed, entry index).  Returns nnz; fills non-NULL arrays. */
int64_t gen_stencil27(int32_t nx, int32_t ny, int32_t nz, int integer_values, uint64_t seed,
                      int32_t *irp, int32_t *icol, double *val)
{
    int64_t n = (int64_t)nx * ny * nz;
    /* Row lengths are products of per-axis spans; the prefix is computed per
     * z-y line so that the fill below can run in parallel. */
    int64_t nnz = 0;
    if (!irp && !icol && !val) {
        for (int32_t z = 0; z < nz; ++z)
            for (int32_t y = 0; y < ny; ++y)
                for (int32_t x = 0; x < nx; ++x)
                    nnz += span3(x, nx) * span3(y, ny) * span3(z, nz);
        return nnz;
    }
    for (int32_t z = 0; z < nz; ++z)
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t x = 0; x < nx; ++x) {
                int64_t i = x + (int64_t)nx * (y + (int64_t)ny * z);
                irp[i] = (int32_t)nnz;
                nnz += span3(x, nx) * span3(y, ny) * span3(z, nz);
            }
    irp[n] = (int32_t)nnz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t x = (int32_t)(i % nx), y = (int32_t)((i / nx) % ny), z = (int32_t)(i / ((int64_t)nx * ny));
        int64_t p = irp[i];
        for (int dz = -1; dz <= 1; ++dz) {
            if (z + dz < 0 || z + dz >= nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                if (y + dy < 0 || y + dy >= ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    if (x + dx < 0 || x + dx >= nx) continue;
                    int64_t j = (x + dx) + (int64_t)nx * ((y + dy) + (int64_t)ny * (z + dz));
                    icol[p] = (int32_t)j;
                    double v;
                    if (j == i)
                        v = integer_values ? 26.0 : 26.0 + unif(seed, ST_VAL, (uint64_t)p);
                    else
                        v = integer_values ? -1.0 : -1.0 + 0.2 * (unif(seed, ST_VAL, (uint64_t)p) - 0.5);
                    val[p] = v;
                    ++p;
                }
            }
        }
    }
    return nnz;
}

/* --------------------------------------------------- row-length drawing */

/* l_i = round(exp(ln(mean) - s^2/2 + s*z_i)) clipped to [lmin, lmax], where
 * z_i is the standard normal for counter i of stream ST_LEN under seed.  The
 * shift -s^2/2 makes `mean` the mean of the unclipped lognormal.  s = 0
 * gives every row round(mean). */
void gen_lognormal_lengths(int32_t n, double mean, double s, int32_t lmin, int32_t lmax,
                           uint64_t seed, int32_t *len)
{
    double mu_log = log(mean) - 0.5 * s * s;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double z = (s == 0.0) ? 0.0 : normal(seed, ST_LEN, (uint64_t)i);
        double l = floor(exp(mu_log + s * z) + 0.5);
        if (l < lmin) l = lmin;
        if (l > lmax) l = lmax;
        len[i] = (int32_t)l;
    }
}

/* Row pointers from row lengths (input construction).  Returns nnz, or -1 if
 * it would not fit an int32 pointer. */
int64_t gen_lengths_to_irp(int32_t n, const int32_t *len, int32_t *irp)
{
    int64_t p = 0;
    for (int32_t i = 0; i < n; ++i) {
        irp[i] = (int32_t)p;
        p += len[i];
        if (p > INT32_MAX) return -1;
    }
    irp[n] = (int32_t)p;
    return p;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Column indices drawn uniformly without replacement inside each row
 * (Floyd's algorithm, with a per-row open-addressing set), then sorted
 * ascending.  Row lengths must not exceed ncols. */
void gen_random_cols(int32_t n, int32_t ncols, const int32_t *irp, uint64_t seed, int32_t *icol)
{
#pragma omp parallel
    {
        int32_t cap = 0;
        int32_t *set = NULL;
#pragma omp for schedule(dynamic, 4096)
        for (int32_t i = 0; i < n; ++i) {
            int32_t k = irp[i + 1] - irp[i];
            if (k == 0) continue;
            int32_t need = 4;
            while (need < 2 * k) need <<= 1;
            if (need > cap) {
                free(set);
                cap = need;
                set = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            }
            for (int32_t t = 0; t < cap; ++t) set[t] = -1;
            int32_t *out = icol + irp[i];
            int32_t m = 0;
            uint64_t base = (uint64_t)i << 32;
            for (int64_t j = (int64_t)ncols - k; j < ncols; ++j) {
                int32_t t = (int32_t)below(seed, ST_COL, base + (uint64_t)(j - (ncols - k)), (uint64_t)j + 1);
                /* insert t if absent, else insert j */
                int32_t cand = t;
                for (int pass = 0; pass < 2; ++pass) {
                    uint32_t h = ((uint32_t)cand * 2654435761u) & (uint32_t)(cap - 1);
                    int found = 0;
                    while (set[h] != -1) {
                        if (set[h] == cand) { found = 1; break; }
                        h = (h + 1) & (uint32_t)(cap - 1);
                    }
                    if (!found) { set[h] = cand; out[m++] = cand; break; }
                    cand = (int32_t)j;
                }
            }
            qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
        }
        free(set);
    }
}

/* Column indices drawn uniformly without replacement from the window
 * [i - w, i + w] (clipped to [0, n-1]) around each row i, then sorted.
 * Row lengths must not exceed the clipped window.  Same counter layout as
 * gen_random_cols. */
void gen_window_cols(int32_t n, int32_t w, const int32_t *irp, uint64_t seed, int32_t *icol)
{
#pragma omp parallel
    {
        int32_t cap = 0;
        int32_t *set = NULL;
#pragma omp for schedule(dynamic, 4096)
        for (int32_t i = 0; i < n; ++i) {
            int32_t k = irp[i + 1] - irp[i];
            if (k == 0) continue;
            int64_t lo = (int64_t)i - w < 0 ? 0 : (int64_t)i - w;
            int64_t hi = (int64_t)i + w > n - 1 ? n - 1 : (int64_t)i + w;
            int64_t span = hi - lo + 1;
            int32_t need = 4;
            while (need < 2 * k) need <<= 1;
            if (need > cap) {
                free(set);
                cap = need;
                set = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            }
            for (int32_t t = 0; t < cap; ++t) set[t] = -1;
            int32_t *out = icol + irp[i];
            int32_t m = 0;
            uint64_t base = (uint64_t)i << 32;
            for (int64_t j = span - k; j < span; ++j) {
                int32_t t = (int32_t)below(seed, ST_COL, base + (uint64_t)(j - (span - k)), (uint64_t)j + 1);
                int32_t cand = t;
                for (int pass = 0; pass < 2; ++pass) {
                    uint32_t h = ((uint32_t)cand * 2654435761u) & (uint32_t)(cap - 1);
                    int found = 0;
                    while (set[h] != -1) {
                        if (set[h] == cand) { found = 1; break; }
                        h = (h + 1) & (uint32_t)(cap - 1);
                    }
                    if (!found) { set[h] = cand; out[m++] = (int32_t)(lo + cand); break; }
                    cand = (int32_t)j;
                }
            }
            qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
        }
        free(set);
    }
}

/* Banded pattern: row i holds columns max(0,i-b) .. min(n-1,i+b).
 * Values U[-1,1) per entry.  Returns nnz; fills non-NULL arrays. */
int64_t gen_banded(int32_t n, int32_t b, uint64_t seed, int32_t *irp, int32_t *icol, double *val)
{
    int64_t p = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t lo = i - b < 0 ? 0 : i - b;
        int32_t hi = i + b > n - 1 ? n - 1 : i + b;
        if (irp) irp[i] = (int32_t)p;
        for (int32_t j = lo; j <= hi; ++j, ++p) {
            if (icol) icol[p] = j;
            if (val) val[p] = -1.0 + 2.0 * unif(seed, ST_VAL, (uint64_t)p);
        }
    }
    if (irp) irp[n] = (int32_t)p;
    return p;
}

/* Uniform draws in [0,1) for an arbitrary stream (job schedules). */
void gen_unif_stream(int64_t m, uint64_t seed, uint64_t stream, double *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = unif(seed, ST_MISC * 1000003ull + stream, (uint64_t)i);
}
