/*
 * ism_oracle.c -- plain, slow, FP64 CPU oracle for the image-source room
 * impulse response (RIR) path and for the source convolution that follows it.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the GPU library; neither side
 * includes or links the other.
 *
 * What is computed (paper section II.A, synthetic dataset generation, which
 * builds RIRs with the image-source method of Allen and Berkley, 1979): every
 * image of the source in a shoebox room, its distance to the microphone, its
 * damping as the product of one reflection coefficient per wall hit times the
 * 1/(4 pi d) spreading law, and its delay d*fs/c split into an integer part and
 * a fractional part.  Each image adds a fractional-delay filter centred on its
 * delay into the RIR.  The paper uses a 7th-order Lagrange filter; the workloads
 * built here use a Hann-windowed sinc, which is evaluated below exactly as
 * defined (no tables, no recurrences, libm sin/cos).
 *
 * Definitions used (where the paper is silent, the reading stated here is
 * the one this project takes):
 *   image (n,l,q in Z; u,v,w in {0,1}):
 *     p = ((1-2u) sx + 2n Lx, (1-2v) sy + 2l Ly, (1-2w) sz + 2q Lz)
 *   wall exponents: x=0 wall |n-u|, x=Lx wall |n|; same for y (l,v), z (q,w);
 *     beta[] order is [x0, xL, y0, yL, z0, zL]
 *   d = |p - r|, tau = d*fs/c, g = prod(beta^e) / (4 pi d)
 *   h(t) = sinc(t) * w(t), sinc(0) = 1,
 *   w(t) = 1/2 (1 + cos(pi t / (K+1))) for |t| < K+1, else 0, K = (taps-1)/2
 *   n0 = floor(tau + 1/2); taps at n = n0 + k, k = -K..K, kept if 0 <= n < len
 *   out[n] = sum over images, in lexicographic (n,l,q,u,v,w) order, of
 *            g * h(n - tau), plain FP64 accumulation.
 *   taps == 8 selects the paper's own filter instead, the 7th-order Lagrange
 *   interpolator: n0 = floor(tau), taps at n = n0 - 3 + j, j = 0..7, with
 *   h_j = prod_{i != j} (D - i) / (j - i), D = tau - (n0 - 3) in [3, 4) (the
 *   delay sits between the two middle taps); time bound n0 - 3 <= len - 1.
 *   Image sets: order_mode 0 (index L1): |n|+|l|+|q| <= N, all 8 parities;
 *               order_mode 1 (reflections): |2n-u|+|2l-v|+|2q-w| <= N;
 *               max_order < 0: every image whose tap support meets [0, len).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math), so
 * that d*d sums and the delay split are plain IEEE double operations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* beta^e by repeated multiplication, so that beta^0 == 1 also for beta == 0 */
static double ipow(double b, long e)
{
    double p = 1.0;
    for (long i = 0; i < e; ++i) p *= b;
    return p;
}

static long labs_l(long a) { return a < 0 ? -a : a; }

/* Hann-windowed sinc fractional-delay kernel h(t) (K = half-length). */
double ism_oracle_fd_tap(double t, int K)
{
    double half = (double)K + 1.0;
    if (fabs(t) >= half) return 0.0;
    double s = (t == 0.0) ? 1.0 : sin(M_PI * t) / (M_PI * t);
    double w = 0.5 * (1.0 + cos(M_PI * t / half));
    return s * w;
}

/* Coefficient j (0..7) of the 7th-order Lagrange fractional-delay interpolator
   at delay D (taps at 0..7): the Lagrange basis polynomial of node j. */
double ism_oracle_lagrange_tap(int j, double D)
{
    double h = 1.0;
    for (int i = 0; i < 8; ++i)
        if (i != j) h *= (D - (double)i) / (double)(j - i);
    return h;
}

/* Image position (closed form of the mirror construction). */
static void image_pos(const double L[3], const double s[3], long n, long l, long q,
                      int u, int v, int w, double p[3])
{
    p[0] = (1 - 2 * u) * s[0] + 2.0 * (double)n * L[0];
    p[1] = (1 - 2 * v) * s[1] + 2.0 * (double)l * L[1];
    p[2] = (1 - 2 * w) * s[2] + 2.0 * (double)q * L[2];
}

static int in_order(long n, long l, long q, int u, int v, int w, int max_order, int mode)
{
    if (max_order < 0) return 1;
    if (mode == 0) return labs_l(n) + labs_l(l) + labs_l(q) <= max_order;
    return labs_l(2 * n - u) + labs_l(2 * l - v) + labs_l(2 * q - w) <= max_order;
}

/*
 * Enumerate images.  Writes up to cap entries of positions (3 doubles) and wall
 * exponents (6 longs as int64) and returns the total number of images of the
 * set (which may exceed cap).  Only for index-bounded sets (max_order >= 0).
 */
long ism_oracle_images(const double L[3], const double src[3], int max_order, int mode,
                       double *pos, int64_t *expo, long cap)
{
    if (max_order < 0) return -1;
    long N = max_order;
    long cnt = 0;
    for (long n = -N - 1; n <= N + 1; ++n)
        for (long l = -N - 1; l <= N + 1; ++l)
            for (long q = -N - 1; q <= N + 1; ++q)
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v)
                        for (int w = 0; w < 2; ++w) {
                            if (!in_order(n, l, q, u, v, w, max_order, mode)) continue;
                            if (cnt < cap) {
                                image_pos(L, src, n, l, q, u, v, w, pos + 3 * cnt);
                                int64_t *e = expo + 6 * cnt;
                                e[0] = labs_l(n - u); e[1] = labs_l(n);
                                e[2] = labs_l(l - v); e[3] = labs_l(l);
                                e[4] = labs_l(q - w); e[5] = labs_l(q);
                            }
                            ++cnt;
                        }
    return cnt;
}

typedef struct {
    long images;      /* images in the enumerated set */
    long contrib;     /* images whose tap support meets [0, len) */
    long taps;        /* (image, k) pairs with 0 <= n0+k < len */
    long max_refl;    /* largest |2n-u|+|2l-v|+|2q-w| among the enumerated images */
} ism_oracle_stats;

/*
 * One RIR (one source, one microphone) into out[0..len) (FP64, overwritten).
 * Returns 0, or -1 on invalid arguments.  stats may be NULL.
 */
int ism_oracle_rir(const double L[3], const double beta[6], const double src[3],
                   const double mic[3], double fs, double c, int max_order, int mode,
                   int len, int taps, double *out, ism_oracle_stats *stats)
{
    const int lag = taps == 8;  /* 7th-order Lagrange; otherwise a windowed sinc */
    if (taps < 1 || (!lag && (taps % 2) == 0) || len < 1 || fs <= 0 || c <= 0) return -1;
    int K = lag ? 4 : (taps - 1) / 2;
    memset(out, 0, sizeof(double) * (size_t)len);
    ism_oracle_stats st = {0, 0, 0, 0};

    /* index box: for the time bound, every image whose first tap is at or before
       len - 1 lies within distance dmax of the microphone (sinc: n0 - K <= len - 1,
       i.e. tau < len - 1 + K + 1/2; Lagrange: floor(tau) - 3 <= len - 1). */
    long bx, by, bz;
    if (max_order >= 0) {
        bx = by = bz = max_order + 1;
    } else {
        double dmax = (lag ? (double)len + 3.0 : (double)len - 1.0 + (double)K + 0.5) * c / fs;
        bx = (long)ceil(dmax / (2.0 * L[0])) + 2;
        by = (long)ceil(dmax / (2.0 * L[1])) + 2;
        bz = (long)ceil(dmax / (2.0 * L[2])) + 2;
    }
    /* taps of an image: n = first .. first + ntap - 1 */
    const int ntap = lag ? 8 : 2 * K + 1;
    for (long n = -bx; n <= bx; ++n)
        for (long l = -by; l <= by; ++l)
            for (long q = -bz; q <= bz; ++q)
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v)
                        for (int w = 0; w < 2; ++w) {
                            if (!in_order(n, l, q, u, v, w, max_order, mode)) continue;
                            double p[3];
                            image_pos(L, src, n, l, q, u, v, w, p);
                            double dx = p[0] - mic[0], dy = p[1] - mic[1], dz = p[2] - mic[2];
                            double d = sqrt(dx * dx + dy * dy + dz * dz);
                            double tau = d * fs / c;
                            long n0 = lag ? (long)floor(tau) : (long)floor(tau + 0.5);
                            long first = lag ? n0 - 3 : n0 - K;
                            if (max_order < 0 && first > len - 1) continue; /* outside the time bound */
                            ++st.images;
                            long refl = labs_l(2 * n - u) + labs_l(2 * l - v) + labs_l(2 * q - w);
                            if (refl > st.max_refl) st.max_refl = refl;
                            if (first + ntap - 1 < 0 || first > len - 1) continue;
                            ++st.contrib;
                            double B = ipow(beta[0], labs_l(n - u)) * ipow(beta[1], labs_l(n)) *
                                       ipow(beta[2], labs_l(l - v)) * ipow(beta[3], labs_l(l)) *
                                       ipow(beta[4], labs_l(q - w)) * ipow(beta[5], labs_l(q));
                            double g = B / (4.0 * M_PI * d);
                            for (int j = 0; j < ntap; ++j) {
                                long idx = first + j;
                                if (idx < 0 || idx >= len) continue;
                                double h = lag ? ism_oracle_lagrange_tap(j, tau - (double)first)
                                               : ism_oracle_fd_tap((double)idx - tau, K);
                                out[idx] += g * h;
                                ++st.taps;
                            }
                        }
    if (stats) *stats = st;
    return 0;
}

/* ---- batch driver over (room, mic) RIRs, threads over RIRs (timing only) ---- */

typedef struct {
    const double *L, *beta, *src, *mics;     /* per room: 3, 6, 3; mics: total x 3 */
    const int32_t *mic_off, *n_mics, *max_order, *rir_len;
    const int64_t *out_off;
    double fs, c; int mode, taps;
    double *out;                              /* FP64 outputs, out_off + m*len */
    const int64_t *rir_list;                  /* flattened (room<<20 | mic) work list */
    long n_list;
    long next;                                /* shared work counter */
    pthread_mutex_t mu;
    long taps_done;
} batch_ctx;

static void *batch_worker(void *arg)
{
    batch_ctx *b = (batch_ctx *)arg;
    long local_taps = 0;
    for (;;) {
        pthread_mutex_lock(&b->mu);
        long i = b->next++;
        pthread_mutex_unlock(&b->mu);
        if (i >= b->n_list) break;
        long room = (long)(b->rir_list[i] >> 20), m = (long)(b->rir_list[i] & 0xFFFFF);
        int len = b->rir_len[room];
        ism_oracle_stats st;
        ism_oracle_rir(b->L + 3 * room, b->beta + 6 * room, b->src + 3 * room,
                       b->mics + 3 * (b->mic_off[room] + m), b->fs, b->c, b->max_order[room],
                       b->mode, len, b->taps, b->out + b->out_off[room] + m * (long)len, &st);
        local_taps += st.taps;
    }
    pthread_mutex_lock(&b->mu);
    b->taps_done += local_taps;
    pthread_mutex_unlock(&b->mu);
    return NULL;
}

/*
 * RIRs listed in rir_list (entries room<<20 | mic), each written at
 * out[out_off[room] + mic*rir_len[room]].  Returns the number of taps, or -1.
 */
long ism_oracle_rir_list(const double *L, const double *beta, const double *src,
                         const double *mics, const int32_t *mic_off, const int32_t *n_mics,
                         const int32_t *max_order, const int32_t *rir_len, const int64_t *out_off,
                         double fs, double c, int mode, int taps, const int64_t *rir_list,
                         long n_list, int nthreads, double *out)
{
    batch_ctx b;
    b.L = L; b.beta = beta; b.src = src; b.mics = mics; b.mic_off = mic_off; b.n_mics = n_mics;
    b.max_order = max_order; b.rir_len = rir_len; b.out_off = out_off; b.fs = fs; b.c = c;
    b.mode = mode; b.taps = taps; b.out = out; b.rir_list = rir_list; b.n_list = n_list;
    b.next = 0; b.taps_done = 0;
    pthread_mutex_init(&b.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, &b);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&b.mu);
    return b.taps_done;
}

/* ---------------- source convolution + sensor noise (paper III.A) ---------------- */

/*
 * One room: y[m][n] = sum_{j=0}^{min(n, hlen-1)} h[m][j] x[n-j] for n < out_len
 * (direct FP64 sum), then, if z is not NULL, y += sigma * z with
 * sigma^2 = P * 10^(-snr_db/10), P = mean of y^2 over all channels and samples
 * of the noiseless signal, z = caller-supplied standard normal deviates
 * [M][out_len].  h is [M][hlen], x is [xlen], y is [M][out_len].
 */
int ism_oracle_conv_room(int M, int hlen, const double *h, int xlen, const double *x,
                         int out_len, double snr_db, const double *z, double *y)
{
    if (M < 1 || hlen < 1 || xlen < 1 || out_len < 1) return -1;
    double P = 0.0;
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < out_len; ++n) {
            double acc = 0.0;
            int jmax = n < hlen - 1 ? n : hlen - 1;
            for (int j = 0; j <= jmax; ++j)
                if (n - j < xlen) acc += h[(size_t)m * hlen + j] * x[n - j];
            y[(size_t)m * out_len + n] = acc;
            P += acc * acc;
        }
    if (!z) return 0;
    P /= (double)M * (double)out_len;
    double sigma = sqrt(P * pow(10.0, -snr_db / 10.0));
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < out_len; ++n)
            y[(size_t)m * out_len + n] += sigma * z[(size_t)m * out_len + n];
    return 0;
}
