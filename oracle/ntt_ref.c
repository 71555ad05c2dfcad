/*
 * Plain C oracle for the BN254-Fr number-theoretic transform.
 *
 * TEST INFRASTRUCTURE ONLY: linked and called by tests/, by the smoke check
 * and by the CPU-baseline leg of the benchmark, never by the library under
 * test. It shares no code, header or table with the GPU path.
 *
 * What it computes (paper: Background, "Number Theory Transformation"):
 * X_k = sum_n x_n w_N^(kn) mod r, w_N = 5^((r-1)/N), natural order in and
 * out, plus the inverse (scaled by N^-1), the coset transform at g*w^k with
 * g = 5, and its inverse. Elements are canonical 4 x 64-bit little-endian
 * limbs in [0, r).
 *
 * Method: a textbook iterative radix-2 decimation-in-time FFT (bit-reversal
 * permutation, then log2(N) butterfly stages). Products mod r use Montgomery
 * multiplication in the coarsely integrated operand scanning form of Koc,
 * Acar and Kaliski (IEEE Micro 1996) with 64-bit words and a 128-bit
 * intermediate. Montgomery constants are derived at start-up from r by
 * repeated modular doubling, not typed in.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC ntt_ref.c -o libntt_ref.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;
typedef struct { uint64_t v[4]; } fe;   /* little-endian limbs */

/* r = 21888242871839275222246405745257275088548364400416034343698204186575808495617 */
static const fe R_MOD = {{0x43E1F593F0000001ULL, 0x2833E84879B97091ULL,
                          0xB85045B68181585DULL, 0x30644E72E131A029ULL}};

static fe MONT_ONE;     /* 2^256 mod r */
static fe MONT_R2;      /* 2^512 mod r */
static uint64_t NPRIME; /* -r^-1 mod 2^64 */
static int initialised = 0;

static int fe_geq(const fe *a, const fe *b) {
    for (int i = 3; i >= 0; --i) {
        if (a->v[i] > b->v[i]) return 1;
        if (a->v[i] < b->v[i]) return 0;
    }
    return 1;
}

static uint64_t fe_sub_raw(fe *out, const fe *a, const fe *b) {
    uint64_t borrow = 0;
    for (int i = 0; i < 4; ++i) {
        u128 d = (u128)a->v[i] - b->v[i] - borrow;
        out->v[i] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
    return borrow;
}

static uint64_t fe_add_raw(fe *out, const fe *a, const fe *b) {
    uint64_t carry = 0;
    for (int i = 0; i < 4; ++i) {
        u128 s = (u128)a->v[i] + b->v[i] + carry;
        out->v[i] = (uint64_t)s;
        carry = (uint64_t)(s >> 64);
    }
    return carry;
}

/* (a + b) mod r for a, b < r */
static fe fe_add(fe a, fe b) {
    fe s, t;
    fe_add_raw(&s, &a, &b);            /* < 2r < 2^256: no carry out */
    if (fe_geq(&s, &R_MOD)) { fe_sub_raw(&t, &s, &R_MOD); return t; }
    return s;
}

/* (a - b) mod r for a, b < r */
static fe fe_sub(fe a, fe b) {
    fe d, t;
    if (fe_sub_raw(&d, &a, &b)) { fe_add_raw(&t, &d, &R_MOD); return t; }
    return d;
}

/* Montgomery product a*b*2^-256 mod r (CIOS), a, b < r. */
static fe mont_mul(fe a, fe b) {
    uint64_t t[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
        uint64_t c = 0;
        for (int j = 0; j < 4; ++j) {
            u128 s = (u128)a.v[j] * b.v[i] + t[j] + c;
            t[j] = (uint64_t)s;
            c = (uint64_t)(s >> 64);
        }
        u128 s = (u128)t[4] + c;
        t[4] = (uint64_t)s;
        t[5] = (uint64_t)(s >> 64);
        uint64_t m = t[0] * NPRIME;
        s = (u128)m * R_MOD.v[0] + t[0];
        c = (uint64_t)(s >> 64);
        for (int j = 1; j < 4; ++j) {
            s = (u128)m * R_MOD.v[j] + t[j] + c;
            t[j - 1] = (uint64_t)s;
            c = (uint64_t)(s >> 64);
        }
        s = (u128)t[4] + c;
        t[3] = (uint64_t)s;
        t[4] = t[5] + (uint64_t)(s >> 64);
    }
    fe out = {{t[0], t[1], t[2], t[3]}};
    if (t[4] || fe_geq(&out, &R_MOD)) { fe o2; fe_sub_raw(&o2, &out, &R_MOD); return o2; }
    return out;
}

static void oracle_init(void) {
    if (initialised) return;
    /* -r^-1 mod 2^64 by Newton iteration x <- x(2 - r x), starting from r
       (valid mod 2^3 for odd r; each step doubles the correct bits). */
    uint64_t r0 = R_MOD.v[0], x = r0;
    for (int i = 0; i < 6; ++i) x *= 2 - r0 * x;
    NPRIME = (uint64_t)0 - x;
    /* 2^256 and 2^512 mod r by doubling 1 repeatedly (each step mod r). */
    fe acc = {{1, 0, 0, 0}};
    for (int i = 0; i < 512; ++i) {
        acc = fe_add(acc, acc);
        if (i == 255) MONT_ONE = acc;
    }
    MONT_R2 = acc;
    initialised = 1;
}

static fe to_mont(fe a) { return mont_mul(a, MONT_R2); }
static fe from_mont(fe a) { fe one = {{1, 0, 0, 0}}; return mont_mul(a, one); }

/* base^e (Montgomery domain in/out), e given as 4 limbs, square and multiply. */
static fe mont_pow(fe base_m, const uint64_t e[4]) {
    fe acc = MONT_ONE;
    for (int i = 255; i >= 0; --i) {
        acc = mont_mul(acc, acc);
        if ((e[i / 64] >> (i % 64)) & 1) acc = mont_mul(acc, base_m);
    }
    return acc;
}

static fe small_mont(uint64_t v) { fe a = {{v, 0, 0, 0}}; return to_mont(a); }

/* w_N = 5^((r-1)/N) in Montgomery form (or its inverse). */
static fe root_mont(int log_n, int inverse) {
    uint64_t e[4];
    fe rm1 = R_MOD; rm1.v[0] -= 1;
    /* (r-1) >> log_n */
    for (int i = 0; i < 4; ++i) {
        uint64_t lo = rm1.v[i] >> log_n;
        uint64_t hi = (i < 3 && log_n) ? (rm1.v[i + 1] << (64 - log_n)) : 0;
        e[i] = lo | hi;
    }
    fe w = mont_pow(small_mont(5), e);
    if (inverse) {
        uint64_t rm2[4] = {R_MOD.v[0] - 2, R_MOD.v[1], R_MOD.v[2], R_MOD.v[3]};
        w = mont_pow(w, rm2);
    }
    return w;
}

static fe inverse_mont(fe a_m) {
    uint64_t rm2[4] = {R_MOD.v[0] - 2, R_MOD.v[1], R_MOD.v[2], R_MOD.v[3]};
    return mont_pow(a_m, rm2);
}

static uint64_t bitrev(uint64_t i, int bits) {
    uint64_t r = 0;
    for (int b = 0; b < bits; ++b) { r = (r << 1) | (i & 1); i >>= 1; }
    return r;
}

/* In-place radix-2 DIT transform of n = 2^log_n Montgomery-form elements. */
static void fft_mont(fe *a, int log_n, int inverse) {
    int64_t n = (int64_t)1 << log_n;
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = (int64_t)bitrev((uint64_t)i, log_n);
        if (i < j) { fe t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    fe *tw = (fe *)malloc(sizeof(fe) * (size_t)(n / 2 > 0 ? n / 2 : 1));
    for (int s = 1; s <= log_n; ++s) {
        int64_t m = (int64_t)1 << s, half = m / 2;
        fe wm = root_mont(s, inverse);
        tw[0] = MONT_ONE;
        for (int64_t j = 1; j < half; ++j) tw[j] = mont_mul(tw[j - 1], wm);
        #pragma omp parallel for schedule(static)
        for (int64_t blk = 0; blk < n / m; ++blk) {
            int64_t start = blk * m;
            for (int64_t j = 0; j < half; ++j) {
                fe u = a[start + j];
                fe v = mont_mul(a[start + j + half], tw[j]);
                a[start + j] = fe_add(u, v);
                a[start + j + half] = fe_sub(u, v);
            }
        }
    }
    free(tw);
}

static int valid_input(const fe *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (fe_geq(&a[i], &R_MOD)) return 0;
    return 1;
}

/*
 * Transform `batch` polynomials of 2^log_n elements each, in place.
 * kind: 0 forward, 1 inverse, 2 coset (g = 5), 3 coset inverse.
 * threads <= 0 keeps the OpenMP default. Returns 0, or -1 on a bad argument
 * or an input element >= r.
 */
int oracle_transform(uint64_t *data, int log_n, int kind, int batch, int threads) {
    if (!data || log_n < 0 || log_n > 28 || kind < 0 || kind > 3 || batch < 0) return -1;
    oracle_init();
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    int64_t n = (int64_t)1 << log_n;
    fe *all = (fe *)data;
    if (!valid_input(all, n * batch)) return -1;
    for (int b = 0; b < batch; ++b) {
        fe *a = all + (int64_t)b * n;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) a[i] = to_mont(a[i]);
        if (kind == 2) {
            /* x_n <- x_n * g^n (sequential powers, then a parallel scale) */
            fe g = small_mont(5), p = MONT_ONE;
            for (int64_t i = 0; i < n; ++i) { a[i] = mont_mul(a[i], p); p = mont_mul(p, g); }
        }
        int inverse = (kind == 1 || kind == 3);
        fft_mont(a, log_n, inverse);
        if (inverse) {
            fe ninv = inverse_mont(small_mont((uint64_t)n));
            #pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) a[i] = mont_mul(a[i], ninv);
        }
        if (kind == 3) {
            fe ginv = inverse_mont(small_mont(5)), p = MONT_ONE;
            for (int64_t i = 0; i < n; ++i) { a[i] = mont_mul(a[i], p); p = mont_mul(p, ginv); }
        }
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) a[i] = from_mont(a[i]);
    }
    return 0;
}

/*
 * One output of the transform from the definition, by Horner's rule over
 * all n inputs: X_k = sum_n x_n z^n with z = w^k (forward), g*w^k (coset),
 * w^-k then scaled by N^-1 (inverse), and additionally by g^-k (coset inverse).
 */
int oracle_eval_output(const uint64_t *x, int log_n, uint64_t k, int kind, uint64_t out[4]) {
    if (!x || !out || log_n < 0 || log_n > 28 || kind < 0 || kind > 3) return -1;
    oracle_init();
    int64_t n = (int64_t)1 << log_n;
    if (k >= (uint64_t)n) return -1;
    const fe *a = (const fe *)x;
    if (!valid_input(a, n)) return -1;
    int inverse = (kind == 1 || kind == 3);
    fe w = root_mont(log_n, inverse);
    uint64_t e[4] = {k, 0, 0, 0};
    fe z = mont_pow(w, e);
    if (kind == 2) z = mont_mul(z, small_mont(5));
    fe acc = {{0, 0, 0, 0}};
    for (int64_t i = n - 1; i >= 0; --i) acc = fe_add(mont_mul(acc, z), to_mont(a[i]));
    if (inverse) acc = mont_mul(acc, inverse_mont(small_mont((uint64_t)n)));
    if (kind == 3) acc = mont_mul(acc, mont_pow(inverse_mont(small_mont(5)), e));
    fe r = from_mont(acc);
    memcpy(out, r.v, sizeof r.v);
    return 0;
}

/* Field product (a*b mod r) on canonical inputs, exposed for pin tests. */
int oracle_mul(const uint64_t a[4], const uint64_t b[4], uint64_t out[4]) {
    oracle_init();
    fe x, y;
    memcpy(x.v, a, sizeof x.v);
    memcpy(y.v, b, sizeof y.v);
    if (fe_geq(&x, &R_MOD) || fe_geq(&y, &R_MOD)) return -1;
    fe p = from_mont(mont_mul(to_mont(x), to_mont(y)));
    memcpy(out, p.v, sizeof p.v);
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
