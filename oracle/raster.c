/*
 * CPU reference (test infrastructure only): tile binning, front-to-back
 * compositing, its backward pass and the instrumented importance blend, in
 * plain float64 loops.  Only the tests, the smoke check and the CPU-baseline
 * timing load this library; the product path never does.
 *
 * Definitions followed:
 *  - Tile-based front-to-back alpha compositing, Appendix A, Eq.
 *    `alpha_compositing`: C(p) = sum_i T_i alpha_i G'_i c_i with
 *    T_i = prod_{j<i} (1 - alpha_j G'_j) over the depth-ordered Gaussians of
 *    the pixel's tile.  Constants (16x16 tiles, alpha = min(0.99, o G'),
 *    skip alpha < 1/255, stop before T would fall below 1e-4) follow the
 *    standard 3DGS rasterizer the paper keeps.
 *  - Importance sweep, Sec. 3.2 "Importance score" and Fig. 3: the
 *    instrumented blend without colour records w_{i,v} = sum_p alpha_p T_p and
 *    the count a_{i,v} of pixels at which g_i is composited.
 *
 * Threads (OpenMP, OMP_NUM_THREADS): pixels are independent in the forward;
 * the backward and the importance blend accumulate per Gaussian, so each
 * thread sums into its own arrays, over an interleaved static share of the
 * image rows, and the per-thread arrays are added in thread order (the same
 * per-term arithmetic; the summation order depends only on the thread count).
 *
 * Layouts: component-major arrays ([2][n] mean2d, [3][n] conic and rgb),
 * images [3][H][W], per-pixel maps [H][W].  Gaussians are visited in list
 * order; the list of a tile is sorted by (tile, float32 depth bits, index).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TILE 16
#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_MIN 1e-4

static int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Tile rectangle [tx0,tx1) x [ty0,ty1) of a Gaussian with integer radius r. */
static void rect_of(double mx, double my, int64_t r, int64_t TX, int64_t TY,
                    int64_t* tx0, int64_t* tx1, int64_t* ty0, int64_t* ty1) {
    int64_t xi = (int64_t)floor(mx), yi = (int64_t)floor(my);
    *tx0 = clampi(floordiv(xi - r, TILE), 0, TX);
    *tx1 = clampi(floordiv(xi + r, TILE) + 1, 0, TX);
    *ty0 = clampi(floordiv(yi - r, TILE), 0, TY);
    *ty1 = clampi(floordiv(yi + r, TILE) + 1, 0, TY);
}

typedef struct {
    uint64_t key;
    uint32_t val;
    int64_t seq;
} pair_t;

static int cmp_pair(const void* pa, const void* pb) {
    const pair_t* a = (const pair_t*)pa;
    const pair_t* b = (const pair_t*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
    return 0;
}

/*
 * Binning.  For every Gaussian i with radius > 0, in ascending i, and every
 * tile of its rectangle in row-major order, emit key = (tile << 32) | bits of
 * the float32 camera depth, value i.  Sort stably by key (ties keep emission
 * order).  Writes min(K, capacity) pairs, the per-tile [start, end) ranges
 * ([2][n_tiles], start row then end row) and returns K.
 */
int64_t gso_bin_sort(int64_t n, const double* mean2d, const int32_t* radius,
                     const float* depth, int32_t width, int32_t height,
                     uint64_t* keys, uint32_t* vals, int64_t capacity,
                     uint32_t* ranges) {
    const int64_t TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    const int64_t n_tiles = TX * TY;
    int64_t K = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (radius[i] <= 0) continue;
        int64_t x0, x1, y0, y1;
        rect_of(mean2d[i], mean2d[n + i], radius[i], TX, TY, &x0, &x1, &y0, &y1);
        K += (x1 - x0) * (y1 - y0);
    }
    for (int64_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
    if (K > capacity || K == 0) return K;
    pair_t* p = (pair_t*)malloc((size_t)K * sizeof(pair_t));
    if (!p) return -1;
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (radius[i] <= 0) continue;
        int64_t x0, x1, y0, y1;
        rect_of(mean2d[i], mean2d[n + i], radius[i], TX, TY, &x0, &x1, &y0, &y1);
        uint32_t dbits;
        memcpy(&dbits, &depth[i], 4);
        for (int64_t ty = y0; ty < y1; ++ty)
            for (int64_t tx = x0; tx < x1; ++tx) {
                p[s].key = ((uint64_t)(ty * TX + tx) << 32) | (uint64_t)dbits;
                p[s].val = (uint32_t)i;
                p[s].seq = s;
                ++s;
            }
    }
    qsort(p, (size_t)K, sizeof(pair_t), cmp_pair);
    for (int64_t k = 0; k < K; ++k) {
        keys[k] = p[k].key;
        vals[k] = p[k].val;
    }
    for (int64_t k = 0; k < K; ++k) {
        int64_t t = (int64_t)(p[k].key >> 32);
        if (k == 0 || (int64_t)(p[k - 1].key >> 32) != t) ranges[t] = (uint32_t)k;
        if (k == K - 1 || (int64_t)(p[k + 1].key >> 32) != t) ranges[n_tiles + t] = (uint32_t)(k + 1);
    }
    free(p);
    return K;
}

static double rel_gap(double v, double thr) { return fabs(v - thr) / thr; }

int gso_num_threads(void) { return omp_get_max_threads(); }

/*
 * Forward compositing of every pixel.  Outputs the colour [3][H][W] (with
 * T_final * bg added), the final transmittance, `last` = 1 + list position of
 * the last composited Gaussian (0 if none), the 1-based list position at which
 * the pixel stopped (or the list length), the smallest relative distance of
 * any threshold test to its threshold (1/255, 0.99, 1e-4) and a hash of every
 * discrete decision taken (which positions were skipped, clamped or stopped).
 */
void gso_render_fwd(int32_t width, int32_t height, int64_t n, const double* mean2d,
                    const double* conic, const double* opacity, const double* rgb,
                    const uint32_t* vals, const uint32_t* ranges, const double* bg,
                    double* out_rgb, double* out_T, uint32_t* out_last,
                    int64_t* out_stop, double* out_margin, uint64_t* out_sig) {
    const int64_t TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    const int64_t n_tiles = TX * TY;
    const int64_t npx = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t v = 0; v < height; ++v)
        for (int64_t u = 0; u < width; ++u) {
            const int64_t t = (v / TILE) * TX + (u / TILE);
            const int64_t start = ranges[t], end = ranges[n_tiles + t];
            const double px = u + 0.5, py = v + 0.5;
            double T = 1.0, C[3] = {0.0, 0.0, 0.0}, margin = INFINITY;
            uint32_t last = 0;
            uint64_t sig = 1469598103934665603ull;
            int64_t stop = end - start;
            for (int64_t k = start; k < end; ++k) {
                const uint32_t j = vals[k];
                const double dx = mean2d[j] - px, dy = mean2d[n + j] - py;
                const double a = conic[j], b = conic[n + j], c = conic[2 * n + j];
                const double power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy;
                const uint64_t pos = (uint64_t)(k - start);
                if (power > 0.0) {
                    sig = (sig ^ (pos * 4 + 0)) * 1099511628211ull;
                    continue;
                }
                const double g = opacity[j] * exp(power);
                const double alpha = g < ALPHA_MAX ? g : ALPHA_MAX;
                double m1 = rel_gap(g, ALPHA_MIN), m2 = rel_gap(g, ALPHA_MAX);
                if (m1 < margin) margin = m1;
                if (m2 < margin) margin = m2;
                if (g > ALPHA_MAX) sig = (sig ^ (pos * 4 + 2)) * 1099511628211ull;
                if (alpha < ALPHA_MIN) {
                    sig = (sig ^ (pos * 4 + 1)) * 1099511628211ull;
                    continue;
                }
                const double Tn = T * (1.0 - alpha);
                double m3 = rel_gap(Tn, T_MIN);
                if (m3 < margin) margin = m3;
                if (Tn < T_MIN) {
                    sig = (sig ^ (pos * 4 + 3)) * 1099511628211ull;
                    stop = k - start + 1;
                    break;
                }
                for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[ch * n + j] * alpha * T;
                T = Tn;
                last = (uint32_t)(k - start + 1);
            }
            const int64_t p = v * width + u;
            for (int ch = 0; ch < 3; ++ch) out_rgb[ch * npx + p] = C[ch] + T * bg[ch];
            out_T[p] = T;
            out_last[p] = last;
            if (out_stop) out_stop[p] = stop;
            if (out_margin) out_margin[p] = margin;
            if (out_sig) out_sig[p] = sig;
        }
    (void)TY;
}

typedef struct {
    uint32_t j;
    double alpha, T, g, G, dx, dy;
} chain_t;

/*
 * Backward of the compositing with the float64 transmittance chain stored per
 * pixel.  With g = dL/dC(p) and the composited Gaussians k of the pixel,
 *   dC/dalpha_k = c_k T_k - (sum_{i>k} c_i alpha_i T_i + T_final bg) / (1 - alpha_k)
 *   dC/dc_k     = alpha_k T_k
 * and alpha = min(0.99, o G), G = exp(power) (zero derivative when clamped).
 * Accumulates (+=) gradients of mean2d [2][n], conic [3][n], opacity [n],
 * rgb [3][n].
 */
void gso_render_bwd(int32_t width, int32_t height, int64_t n, const double* mean2d,
                    const double* conic, const double* opacity, const double* rgb,
                    const uint32_t* vals, const uint32_t* ranges, const double* bg,
                    const double* grad_img, double* d_mean2d, double* d_conic,
                    double* d_opacity, double* d_rgb) {
    const int64_t TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    const int64_t n_tiles = TX * TY;
    const int64_t npx = (int64_t)width * height;
    int64_t max_len = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
        int64_t l = (int64_t)ranges[n_tiles + t] - (int64_t)ranges[t];
        if (l > max_len) max_len = l;
    }
    const int nt = omp_get_max_threads();
    /* per-thread accumulators: 9 rows of n (mean2d 2, conic 3, opacity 1, rgb 3) */
    double* priv = nt > 1 ? (double*)calloc((size_t)nt * 9 * (size_t)n, sizeof(double)) : NULL;
#pragma omp parallel num_threads(nt)
    {
    const int tid = omp_get_thread_num();
    double* acc = priv ? priv + (size_t)tid * 9 * (size_t)n : NULL;
    double* d_mean2d_t = acc ? acc : d_mean2d;
    double* d_conic_t = acc ? acc + 2 * n : d_conic;
    double* d_opacity_t = acc ? acc + 5 * n : d_opacity;
    double* d_rgb_t = acc ? acc + 6 * n : d_rgb;
    chain_t* ch = (chain_t*)malloc((size_t)(max_len + 1) * sizeof(chain_t));
#pragma omp for schedule(static, 1)
    for (int64_t v = 0; v < height; ++v)
        for (int64_t u = 0; u < width; ++u) {
            const int64_t t = (v / TILE) * TX + (u / TILE);
            const int64_t start = ranges[t], end = ranges[n_tiles + t];
            const double px = u + 0.5, py = v + 0.5;
            double T = 1.0;
            int64_t m = 0;
            for (int64_t k = start; k < end; ++k) {
                const uint32_t j = vals[k];
                const double dx = mean2d[j] - px, dy = mean2d[n + j] - py;
                const double a = conic[j], b = conic[n + j], c = conic[2 * n + j];
                const double power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy;
                if (power > 0.0) continue;
                const double G = exp(power);
                const double g = opacity[j] * G;
                const double alpha = g < ALPHA_MAX ? g : ALPHA_MAX;
                if (alpha < ALPHA_MIN) continue;
                const double Tn = T * (1.0 - alpha);
                if (Tn < T_MIN) break;
                ch[m].j = j; ch[m].alpha = alpha; ch[m].T = T; ch[m].g = g; ch[m].G = G;
                ch[m].dx = dx; ch[m].dy = dy;
                ++m;
                T = Tn;
            }
            const double Tfin = T;
            const int64_t p = v * width + u;
            const double gi[3] = {grad_img[p], grad_img[npx + p], grad_img[2 * npx + p]};
            double suffix[3] = {0.0, 0.0, 0.0};  /* sum_{i>k} c_i alpha_i T_i */
            for (int64_t q = m - 1; q >= 0; --q) {
                const chain_t* e = &ch[q];
                const uint32_t j = e->j;
                double dl_dalpha = 0.0;
                for (int c3 = 0; c3 < 3; ++c3) {
                    const double cj = rgb[c3 * n + j];
                    const double dc = cj * e->T - (suffix[c3] + Tfin * bg[c3]) / (1.0 - e->alpha);
                    dl_dalpha += gi[c3] * dc;
                    d_rgb_t[c3 * n + j] += gi[c3] * e->alpha * e->T;
                }
                for (int c3 = 0; c3 < 3; ++c3) suffix[c3] += rgb[c3 * n + j] * e->alpha * e->T;
                if (e->g > ALPHA_MAX) continue;  /* clamped: alpha is constant */
                const double dl_dG = dl_dalpha * opacity[j];
                d_opacity_t[j] += dl_dalpha * e->G;
                const double dl_dpower = dl_dG * e->G;
                const double a = conic[j], b = conic[n + j], c = conic[2 * n + j];
                d_mean2d_t[j] += dl_dpower * (-(a * e->dx + b * e->dy));
                d_mean2d_t[n + j] += dl_dpower * (-(b * e->dx + c * e->dy));
                d_conic_t[j] += dl_dpower * (-0.5 * e->dx * e->dx);
                d_conic_t[n + j] += dl_dpower * (-e->dx * e->dy);
                d_conic_t[2 * n + j] += dl_dpower * (-0.5 * e->dy * e->dy);
            }
        }
    free(ch);
    }
    if (priv) {
        double* outs[9] = {d_mean2d, d_mean2d + n, d_conic, d_conic + n, d_conic + 2 * n, d_opacity,
                           d_rgb, d_rgb + n, d_rgb + 2 * n};
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int r = 0; r < 9; ++r)
                for (int t = 0; t < nt; ++t) outs[r][j] += priv[((size_t)t * 9 + r) * (size_t)n + j];
        free(priv);
    }
    (void)TY;
}

/*
 * Instrumented blend without colour for one view: for each pixel and each
 * Gaussian composited at it, w[j] += alpha T (T before compositing j) and
 * a[j] += 1.  Accumulates into w and a.  With footprint = 1, a[j] instead
 * counts every pixel of j's tiles inside its footprint (the kernel value
 * passes the 1/255 test), composited or not: occluded pixels and pixels that
 * stopped earlier count too (w is unchanged).
 */
void gso_importance_blend(int32_t width, int32_t height, int64_t n, const double* mean2d,
                          const double* conic, const double* opacity, const uint32_t* vals,
                          const uint32_t* ranges, double* w, int64_t* a, int32_t footprint) {
    const int64_t TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    const int64_t n_tiles = TX * TY;
    const int nt = omp_get_max_threads();
    double* wp = nt > 1 ? (double*)calloc((size_t)nt * (size_t)n, sizeof(double)) : NULL;
    int64_t* ap = nt > 1 ? (int64_t*)calloc((size_t)nt * (size_t)n, sizeof(int64_t)) : NULL;
#pragma omp parallel num_threads(nt)
    {
    const int tid = omp_get_thread_num();
    double* w_t = wp ? wp + (size_t)tid * (size_t)n : w;
    int64_t* a_t = ap ? ap + (size_t)tid * (size_t)n : a;
#pragma omp for schedule(static, 1)
    for (int64_t v = 0; v < height; ++v)
        for (int64_t u = 0; u < width; ++u) {
            const int64_t t = (v / TILE) * TX + (u / TILE);
            const int64_t start = ranges[t], end = ranges[n_tiles + t];
            const double px = u + 0.5, py = v + 0.5;
            double T = 1.0;
            int stopped = 0;
            for (int64_t k = start; k < end; ++k) {
                const uint32_t j = vals[k];
                const double dx = mean2d[j] - px, dy = mean2d[n + j] - py;
                const double a_ = conic[j], b_ = conic[n + j], c_ = conic[2 * n + j];
                const double power = -0.5 * (a_ * dx * dx + c_ * dy * dy) - b_ * dx * dy;
                if (power > 0.0) continue;
                const double g = opacity[j] * exp(power);
                const double alpha = g < ALPHA_MAX ? g : ALPHA_MAX;
                if (alpha < ALPHA_MIN) continue;
                if (footprint) a_t[j] += 1;
                if (stopped) continue;
                const double Tn = T * (1.0 - alpha);
                if (Tn < T_MIN) {
                    if (!footprint) break;
                    stopped = 1;
                    continue;
                }
                w_t[j] += alpha * T;
                if (!footprint) a_t[j] += 1;
                T = Tn;
            }
        }
    }
    if (wp) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int t = 0; t < nt; ++t) {
                w[j] += wp[(size_t)t * (size_t)n + j];
                a[j] += ap[(size_t)t * (size_t)n + j];
            }
        free(wp);
        free(ap);
    }
    (void)TY;
}
