/*
 * oracle.c -- plain, slow, single-threaded FP64 reference for the run-time
 * CRS transformation method of Katagiri & Sato, "An Auto-tuning Method for
 * Run-time Data Transformation for Sparse Matrix-Vector Multiplication"
 * (arXiv:2407.00019).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no code with the
 * GPU library and includes no HIP header.  Build: gcc -O2 -ffp-contract=off
 * (no fused multiply-add, no fast-math), so every floating-point operation
 * below is one IEEE-754 binary64 operation in the order written.
 *
 * Conventions.  Indices are 0-based: the paper's IRP(1)=1 ... IRP(N+1)=NNZ+1
 * becomes irp[0]=0 ... irp[n]=nnz.  Every matrix is square, n x n (section
 * 2.1).  Values are handled as opaque elements of `vbytes` bytes in the
 * transformations (they are moved, never computed on) and as binary64 in the
 * SpMV loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ input */

/* Checks the CRS contract (section 2.1): irp[0] = 0, irp[n] = nnz, irp
 * non-decreasing, 0 <= icol[p] < n.  Returns 0 when valid, else a bit mask:
 * 1 irp[0] != 0, 2 irp[n] != nnz, 4 irp decreasing somewhere, 8 a column out
 * of range. */
int orc_validate_crs(int32_t n, int64_t nnz, const int32_t *irp, const int32_t *icol)
{
    int bad = 0;
    if (irp[0] != 0) bad |= 1;
    if ((int64_t)irp[n] != nnz) bad |= 2;
    for (int32_t i = 0; i < n; ++i)
        if (irp[i + 1] < irp[i]) bad |= 4;
    if (!(bad & 6))
        for (int64_t p = 0; p < nnz; ++p)
            if (icol[p] < 0 || icol[p] >= n) bad |= 8;
    return bad;
}

/* ------------------------------------------------------ D_mat, Eq. (4) */

/* Row-length moments: l_i = irp[i+1] - irp[i] counts every stored entry of
 * row i.  s1 = sum l_i, s2 = sum l_i^2 (exact integers), and the largest and
 * smallest l_i. */
void orc_row_moments(int32_t n, const int32_t *irp, int64_t *s1, int64_t *s2,
                     int32_t *lmax, int32_t *lmin)
{
    int64_t a = 0, b = 0;
    int32_t hi = 0, lo = INT32_MAX;
    for (int32_t i = 0; i < n; ++i) {
        int64_t l = (int64_t)irp[i + 1] - irp[i];
        a += l;
        b += l * l;
        if (l > hi) hi = (int32_t)l;
        if (l < lo) lo = (int32_t)l;
    }
    *s1 = a;
    *s2 = b;
    *lmax = hi;
    *lmin = (n > 0) ? lo : 0;
}

/* Locality of a CRS matrix (a cost-model feature, not part of the paper):
 * the matrix bandwidth, the largest |i - j| over every stored entry a_ij
 * (0 when there is none). */
int32_t orc_bandwidth(int32_t n, const int32_t *irp, const int32_t *icol)
{
    int64_t w = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = irp[i]; p < irp[i + 1]; ++p) {
            int64_t d = (int64_t)icol[p] - i;
            if (d < 0) d = -d;
            if (d > w) w = d;
        }
    }
    return (int32_t)w;
}

/* Nearest binary64 to a non-negative 128-bit integer, ties to even. */
double orc_u128_to_double(uint64_t hi, uint64_t lo)
{
    unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;
    int bits = 0;
    for (unsigned __int128 t = v; t; t >>= 1) ++bits;
    if (bits <= 53) return (double)(uint64_t)v;
    int shift = bits - 53;
    unsigned __int128 mant = v >> shift;
    unsigned __int128 rem = v - (mant << shift);
    unsigned __int128 half = (unsigned __int128)1 << (shift - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    return ldexp((double)(uint64_t)mant, shift);
}

/* Eq. (4): D_mat = sigma / mu over the row lengths, with mu their mean and
 * sigma their (population) standard deviation.  With
 * num = n*s2 - s1^2 (exact, = n^2 sigma^2):
 *   mu = s1 / n,  sigma = sqrt(num) / n,  D_mat = sqrt(num) / s1,
 * each operation rounded once; num itself is rounded once to binary64.
 * An empty matrix (s1 = 0) has D_mat = 0. */
void orc_dmat(int32_t n, int64_t s1, int64_t s2, double *mu, double *sigma, double *d)
{
    unsigned __int128 num = (unsigned __int128)(uint64_t)n * (uint64_t)s2
                          - (unsigned __int128)(uint64_t)s1 * (uint64_t)s1;
    double r = sqrt(orc_u128_to_double((uint64_t)(num >> 64), (uint64_t)num));
    *mu = (double)s1 / (double)n;
    *sigma = r / (double)n;
    *d = (s1 == 0) ? 0.0 : r / (double)s1;
}

/* ------------------------------------------------ COO expansion, sec. 2.1 */

/* COO-Row: IROW(p) is the row that owns position p; the row pointer gives
 * each row's first position.  The same expansion of the CCS column pointer
 * gives the column index of COO-Column (Phase II).  `ptr` has n+1 entries. */
void orc_expand_ptr(int32_t n, const int32_t *ptr, int32_t *idx)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
            idx[p] = i;
}

/* -------------------------------------------- CRS -> CCS, Phase I (sec 2.1)
 *
 * Written from what the column-wise form is, not from the loop that builds
 * it.  CCS holds the same entries grouped by column: ccp[j] is the number of
 * entries whose column is below j (so ccp[0] = 0 and ccp[n] = nnz), and the
 * entries of column j fill positions ccp[j] .. ccp[j+1]-1 in the order the
 * rows give them -- by row, and within a row by storage position, the order
 * the paper's walk over the rows produces.  CRS position p grows with the
 * row and with the place inside the row, so the key (icol[p], p) of every
 * entry is distinct and sorting the keys ascending yields exactly that
 * order; irow_t takes the row that owns each position and val_t its value.
 * Out-of-place: the CRS arrays are left untouched. */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

int orc_csr_to_ccs(int32_t n, const int32_t *irp, const int32_t *icol,
                   const void *val, int vbytes,
                   int32_t *ccp, int32_t *irow_t, void *val_t)
{
    int64_t nnz = irp[n];
    uint64_t *key = malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *row_of = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!key || !row_of) {
        free(key);
        free(row_of);
        return -1;
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = irp[i]; p < irp[i + 1]; ++p)
            row_of[p] = i;
    for (int64_t p = 0; p < nnz; ++p)
        key[p] = ((uint64_t)(uint32_t)icol[p] << 32) | (uint64_t)p;
    qsort(key, (size_t)nnz, sizeof(uint64_t), cmp_u64);
    const unsigned char *v = (const unsigned char *)val;
    unsigned char *vt = (unsigned char *)val_t;
    for (int64_t q = 0; q < nnz; ++q) {
        int64_t p = (int64_t)(key[q] & 0xffffffffu);
        irow_t[q] = row_of[p];
        memcpy(vt + (size_t)q * vbytes, v + (size_t)p * vbytes, (size_t)vbytes);
    }
    int64_t q = 0;
    for (int32_t j = 0; j <= n; ++j) {
        while (q < nnz && (int64_t)(key[q] >> 32) < j) ++q;
        ccp[j] = (int32_t)q;
    }
    free(key);
    free(row_of);
    return 0;
}

/* ------------------------------------------------------ ELL, section 2.1
 *
 * Widest compressed line: the ELL width nz (the paper's "bandwidth length")
 * is the largest number of stored entries in one row (one column for the
 * column-wise form). */
int32_t orc_max_len(int32_t n, const int32_t *ptr)
{
    int32_t w = 0;
    for (int32_t i = 0; i < n; ++i)
        if (ptr[i + 1] - ptr[i] > w) w = ptr[i + 1] - ptr[i];
    return w;
}

/* Packs a compressed-line matrix (ptr/idx/val: CRS rows, or CCS columns)
 * into ELL with `width` slots per line.  The arrays are the paper's
 * VAL(1:n,1:nz) in Fortran order, so slot k of line i sits at k*n + i
 * (the J_PTR = N*(K-1)+I addressing of Fig. 3).  Slots past a line's length
 * are padding: value +0.0 (all bits zero) and index i, the line's own index.
 * Stored entries keep their order within the line. */
void orc_to_ell(int32_t n, const int32_t *ptr, const int32_t *idx, const void *val, int vbytes,
                int32_t width, void *ell_val, int32_t *ell_idx)
{
    const unsigned char *v = (const unsigned char *)val;
    unsigned char *ev = (unsigned char *)ell_val;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = ptr[i + 1] - ptr[i];
        for (int32_t k = 0; k < width; ++k) {
            int64_t s = (int64_t)k * n + i;
            if (k < len) {
                ell_idx[s] = idx[ptr[i] + k];
                memcpy(ev + (size_t)s * vbytes, v + (size_t)(ptr[i] + k) * vbytes, (size_t)vbytes);
            } else {
                ell_idx[s] = i;
                memset(ev + (size_t)s * vbytes, 0, (size_t)vbytes);
            }
        }
    }
}

/* ------------------------------------------------------------------- SpMV
 *
 * y = A x in binary64.  y is cleared to +0.0 first, then each product is
 * added in the loop order of the paper's figures run with one thread. */

/* CRS: rows in order, each row's entries in storage order. */
void orc_spmv_crs(int32_t n, const int32_t *irp, const int32_t *icol, const double *val,
                  const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = irp[i]; p < irp[i + 1]; ++p)
            s = s + val[p] * x[icol[p]];
        y[i] = s;
    }
}

/* COO-Row (Fig. 2 with one thread): positions in storage order,
 * y(row) += val * x(col). */
void orc_spmv_coo_row(int32_t n, int64_t nnz, const int32_t *irow, const int32_t *icol,
                      const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t p = 0; p < nnz; ++p)
        y[irow[p]] = y[irow[p]] + val[p] * x[icol[p]];
}

/* ELL-Row (Fig. 3): slots k outer, rows i inner; padding slots included. */
void orc_spmv_ell_row(int32_t n, int32_t width, const double *ell_val, const int32_t *ell_col,
                      const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int32_t k = 0; k < width; ++k)
        for (int32_t i = 0; i < n; ++i) {
            int64_t s = (int64_t)k * n + i;
            y[i] = y[i] + ell_val[s] * x[ell_col[s]];
        }
}

/* COO-Column (Fig. 1 with one thread): entries in column order,
 * y(row) += val * x(col). */
void orc_spmv_coo_col(int32_t n, int64_t nnz, const int32_t *jcol, const int32_t *irow_t,
                      const double *val_t, const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t q = 0; q < nnz; ++q)
        y[irow_t[q]] = y[irow_t[q]] + val_t[q] * x[jcol[q]];
}

/* ELL-Column: columns j outer, slots k inner, y(row(j,k)) += val * x(j);
 * the same per-row addition order as COO-Column. */
void orc_spmv_ell_col(int32_t n, int32_t width, const double *ell_val, const int32_t *ell_row,
                      const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int32_t j = 0; j < n; ++j)
        for (int32_t k = 0; k < width; ++k) {
            int64_t s = (int64_t)k * n + j;
            y[ell_row[s]] = y[ell_row[s]] + ell_val[s] * x[j];
        }
}

/* -------------------------------------------------- reduced-precision values
 *
 * Not part of the paper.  Values are rounded once from binary64 to the
 * storage format, to nearest with ties to even, straight from the binary64
 * value (no intermediate binary32 step).  Formats: p significand bits
 * (including the hidden one), emin the smallest normal exponent, emax the
 * largest.  binary32: p 24, emin -126, emax 127.  bfloat16: p 8, emin -126,
 * emax 127.  binary16: p 11, emin -14, emax 15.  Finite inputs only. */

/* Rounds v to the format and returns the rounded value as binary64
 * (+-inf on overflow). */
static double round_to_format(double v, int p, int emin, int emax)
{
    if (v == 0.0 || isnan(v) || isinf(v)) return v;
    int e;
    frexp(v, &e);             /* |v| = m 2^e, m in [0.5, 1): exponent of v is e-1 */
    int ex = e - 1;
    if (ex < emin) ex = emin; /* subnormal range: fixed quantum 2^(emin-p+1) */
    int qexp = ex - (p - 1);  /* quantum of the binade */
    double q = ldexp(v, -qexp);          /* exact */
    double r = ldexp(nearbyint(q), qexp); /* nearbyint rounds half to even */
    double maxv = ldexp(2.0 - ldexp(1.0, 1 - p), emax);
    if (fabs(r) > maxv) return copysign(INFINITY, v);
    return r;
}

/* Encodes a value already representable in the format into its bits. */
static uint32_t encode_format(double r, int p, int emin, int ebits)
{
    uint32_t sign = signbit(r) ? 1u : 0u;
    int mbits = p - 1;
    uint32_t bias = (1u << (ebits - 1)) - 1;
    uint32_t out;
    if (isinf(r)) {
        out = ((1u << ebits) - 1u) << mbits;
    } else if (r == 0.0) {
        out = 0;
    } else {
        int e;
        frexp(r, &e);
        int ex = e - 1;
        if (ex < emin) {      /* subnormal: biased exponent 0 */
            out = (uint32_t)ldexp(fabs(r), -(emin - mbits));
        } else {
            uint32_t frac = (uint32_t)(ldexp(fabs(r), mbits - ex) - ldexp(1.0, mbits));
            out = ((uint32_t)(ex + (int)bias) << mbits) | frac;
        }
    }
    return (sign << (ebits + mbits)) | out;
}

/* dtype: 1 binary32, 2 bfloat16, 3 binary16.  Writes m elements of 4 or 2
 * bytes. */
void orc_round_values(int dtype, int64_t m, const double *in, void *out)
{
    for (int64_t t = 0; t < m; ++t) {
        if (dtype == 1) {
            double r = round_to_format(in[t], 24, -126, 127);
            uint32_t b = encode_format(r, 24, -126, 8);
            memcpy((unsigned char *)out + 4 * t, &b, 4);
        } else if (dtype == 2) {
            double r = round_to_format(in[t], 8, -126, 127);
            uint16_t b = (uint16_t)encode_format(r, 8, -126, 8);
            memcpy((unsigned char *)out + 2 * t, &b, 2);
        } else {
            double r = round_to_format(in[t], 11, -14, 15);
            uint16_t b = (uint16_t)encode_format(r, 11, -14, 5);
            memcpy((unsigned char *)out + 2 * t, &b, 2);
        }
    }
}

/* Exact widening of stored values back to binary64. */
void orc_widen_values(int dtype, int64_t m, const void *in, double *out)
{
    for (int64_t t = 0; t < m; ++t) {
        uint32_t b;
        int mbits, ebits, emin;
        if (dtype == 1) {
            memcpy(&b, (const unsigned char *)in + 4 * t, 4);
            mbits = 23; ebits = 8; emin = -126;
        } else {
            uint16_t h;
            memcpy(&h, (const unsigned char *)in + 2 * t, 2);
            b = h;
            if (dtype == 2) { mbits = 7; ebits = 8; emin = -126; }
            else            { mbits = 10; ebits = 5; emin = -14; }
        }
        uint32_t sign = (b >> (mbits + ebits)) & 1u;
        uint32_t ef = (b >> mbits) & ((1u << ebits) - 1u);
        uint32_t frac = b & ((1u << mbits) - 1u);
        double v;
        if (ef == 0)
            v = ldexp((double)frac, emin - mbits);
        else if (ef == (1u << ebits) - 1u)
            v = frac ? NAN : INFINITY;
        else
            v = ldexp((double)((1u << mbits) | frac), (int)ef - ((1 << (ebits - 1)) - 1) - mbits);
        out[t] = sign ? -v : v;
    }
}
