/*
 * oracle/raster.c -- plain FP64 CPU reference for ordered splat compositing and its gradients.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load this library. The product path (the HIP library) never calls it, and the two share no
 * code, header, table or constant.
 *
 * What it computes, per pixel u with centre (x + 0.5, y + 0.5), over the splats in the given
 * depth order (Sec. 2.1.2):
 *   alpha_i = min(alpha_max, o_i exp(-q_i / 2)),  q_i = d^T Q_i d,  d = u - mu_i,
 *   Q_i = [[a, b], [b, c]] (the conic, inverse 2D covariance);
 *   fragments with alpha_i < alpha_min are discarded in both passes (Sec. 2.1.2, threshold 1/255);
 *   forward: T_1 = 1, C = sum_i T_i alpha_i c_i, T_{i+1} = T_i (1 - alpha_i)        (Eq. 2, Eq. 5)
 *     (optional forward T-culling: a fragment with T_i < t_min_fwd is skipped, Sec. 2.1.4);
 *   backward (Procedure 1, ComputeGradient): state (C'_1, T_1) = (C, 1); per fragment in the same
 *     order: cull if alpha_i < alpha_min; cull if T_i < t_min_bwd (the state is then left as is);
 *     otherwise dL/dc_i = dL/dC alpha_i T_i                                         (Eq. 3)
 *               dL/dalpha_i = dL/dC . (c_i T_i - C'_i) / (1 - alpha_i)              (Eq. 7)
 *               (C'_{i+1}, T_{i+1}) = (C'_i - T_i alpha_i c_i, T_i (1 - alpha_i))   (Eqs. 5, 6)
 *     and the chain rule to theta_i = (mu, conic, o, c) (the bwd_diff step): through a clamped
 *     alpha the gradient to (o, q) is zero; d alpha/d o = exp(-q/2); d alpha/d q = -alpha/2;
 *     dq/da = dx^2, dq/db = 2 dx dy, dq/dc = dy^2, dq/dmu = -2 Q d.
 *
 * Extension beyond Eq. 2 (zero by default): a background colour bg seen through the final
 * transmittance, C += T_final bg, which C'_1 = C carries into the backward unchanged; and a
 * gradient dL/dT_final, which adds -dL/dT_final T_final / (1 - alpha_i) to dL/dalpha_i (the
 * derivative of T_final = prod (1 - alpha_j)), with dL/dbg = sum over pixels dL/dC T_final.
 *
 * Mixed-precision emulation (Sec. 3.3): with `emulate` set, the stored per-pixel state (colour
 * and T) is rounded to the framebuffer format either after every fragment store (render-target
 * semantics) or only when the pixel's state is written back at rest; arithmetic stays FP64.
 * In the unorm formats the splat colour is saturated to [0, 1] (Sec. 3.3).
 *
 * Ambiguity flags: a decision the FP32 GPU path could take the other way is counted per pixel:
 * the alpha threshold test when |q - r^2| lies inside a band set by the magnitude of q's terms,
 * T tests when |T / t_min - 1| <= tau, and the alpha clamp when alpha_raw is within the band of
 * alpha_max. Exact comparisons of counts are made only at pixels with no such decision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OF_F32 = 0, OF_F16 = 1, OF_UNORM16 = 2, OF_BF16 = 3, OF_UNORM8 = 4 };

typedef struct {
    double alpha_min, alpha_max, t_min_fwd, t_min_bwd;
    double beta;      /* alpha-test band, relative to |a|dx^2 + 2|b dx dy| + |c|dy^2 + r^2 */
    double beta_abs;  /* alpha-test band, absolute, on q */
    double tau;       /* T-test band, relative */
    int32_t fb_format;
    int32_t emulate;   /* 0: pure FP64; 1: round the stored state to fb_format */
    int32_t fb_round;  /* 0: at rest; 1: after every fragment store */
    int32_t saturate;  /* clamp the splat colour to <= 1 */
    int32_t prefilter; /* 0: every splat at every pixel; 1: skip splats whose exact alpha>=alpha_min
                          ellipse bounding box excludes the pixel centre */
    int32_t nthreads;
    double background[3]; /* colour behind the last splat: C += T_final bg (0: Eq. 2 as printed) */
} ocfg_t;

/* ---- format rounding (round to nearest, ties to even, from FP64) ------------------------- */

/* Round |x| to a binary format with `mant` fraction bits and minimum normal exponent `emin`. */
static double round_binary(double x, int mant, int emin, double maxfinite)
{
    if (x == 0.0 || !isfinite(x)) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e);          /* ax = m 2^e, m in [0.5, 1): leading bit has weight 2^(e-1) */
    int lead = e - 1;
    if (lead < emin) lead = emin;                 /* subnormal range: fixed spacing */
    double ulp = ldexp(1.0, lead - mant);
    double r = nearbyint(ax / ulp) * ulp;         /* default rounding mode: ties to even */
    if (r > maxfinite) r = INFINITY;
    return copysign(r, x);
}

static double round_unorm(double x, double levels)
{
    if (!(x > 0.0)) return 0.0;                   /* also maps NaN to 0 */
    if (x > 1.0) x = 1.0;
    return nearbyint(x * levels) / levels;
}

double oracle_round_fmt(double x, int32_t fmt)
{
    switch (fmt) {
    case OF_F32: return (double)(float)x;
    case OF_F16: return round_binary(x, 10, -14, 65504.0);
    case OF_BF16: return round_binary(x, 7, -126, 3.3895313892515355e38);
    case OF_UNORM16: return round_unorm(x, 65535.0);
    case OF_UNORM8: return round_unorm(x, 255.0);
    default: return x;
    }
}

void oracle_round_array(double* x, int64_t count, int32_t fmt)
{
    for (int64_t i = 0; i < count; ++i) x[i] = oracle_round_fmt(x[i], fmt);
}

/* ---- one fragment's alpha ----------------------------------------------------------------- */

typedef struct {
    double dx, dy, q, e, araw, alpha;
    int amb;   /* alpha-threshold decision inside the band */
} frag_t;

static void eval_fragment(const ocfg_t* cfg, double px, double py, const double* m,
                          const double* cn, double o, frag_t* f)
{
    double a = cn[0], b = cn[1], c = cn[2];
    f->dx = px - (double)m[0];
    f->dy = py - (double)m[1];
    double t1 = a * f->dx * f->dx, t2 = 2.0 * b * f->dx * f->dy, t3 = c * f->dy * f->dy;
    f->q = t1 + t2 + t3;
    f->e = exp(-0.5 * f->q);
    f->araw = o * f->e;
    f->alpha = f->araw < cfg->alpha_max ? f->araw : cfg->alpha_max;
    f->amb = 0;
    if (o > 0.0) {
        double r2 = 2.0 * log(o / cfg->alpha_min);   /* alpha_raw >= alpha_min  <=>  q <= r2 */
        double band = cfg->beta * (fabs(t1) + fabs(t2) + fabs(t3) + fabs(r2)) + cfg->beta_abs;
        if (fabs(f->q - r2) <= band) f->amb = 1;
    }
}

/* ---- conservative per-splat pixel ranges (pure skipping of alpha < alpha_min pixels) ------ */

typedef struct { int32_t x0, x1, y0, y1; int32_t any; } range_t;

static void splat_range(const ocfg_t* cfg, const double* m, const double* cn, double o, range_t* r)
{
    double a = cn[0], b = cn[1], c = cn[2];
    double det = a * c - b * b;
    r->any = 1;
    if (!(a > 0.0 && c > 0.0 && det > 0.0)) {   /* unbounded support: never skipped */
        r->x0 = INT32_MIN / 2; r->x1 = INT32_MAX / 2; r->y0 = INT32_MIN / 2; r->y1 = INT32_MAX / 2;
        return;
    }
    if (!(o >= cfg->alpha_min)) { r->any = 0; return; }   /* q >= 0 so alpha <= o < alpha_min */
    double r2 = 2.0 * log(o / cfg->alpha_min);
    double hx = sqrt(r2 * c / det) * (1.0 + 1e-9) + 1e-9;
    double hy = sqrt(r2 * a / det) * (1.0 + 1e-9) + 1e-9;
    double lx = floor((double)m[0] - hx - 0.5), ux = ceil((double)m[0] + hx - 0.5);
    double ly = floor((double)m[1] - hy - 0.5), uy = ceil((double)m[1] + hy - 0.5);
    const double big = 1e9;
    r->x0 = (int32_t)fmax(fmin(lx, big), -big);
    r->x1 = (int32_t)fmax(fmin(ux, big), -big);
    r->y0 = (int32_t)fmax(fmin(ly, big), -big);
    r->y1 = (int32_t)fmax(fmin(uy, big), -big);
}

/* ---- the raster --------------------------------------------------------------------------- */

int oracle_raster(const ocfg_t* cfg, int32_t n, const double* means2d, const double* conics,
                  const double* opac, const double* rgb, const int32_t* order, int32_t n_order,
                  int32_t W, int32_t H, int32_t x0, int32_t y0, int32_t cw, int32_t ch,
                  const double* dL_dimg, double* out_img, double* out_T, int32_t* out_cov,
                  int32_t* out_live, int32_t* out_amb, double* grad, const double* dL_dT,
                  double* grad_bg)
{
    if (n < 0 || n_order < 0 || W <= 0 || H <= 0 || cw < 0 || ch < 0) return 1;
    if (x0 < 0 || y0 < 0 || x0 + cw > W || y0 + ch > H) return 1;
    for (int32_t k = 0; k < n_order; ++k)
        if (order[k] < 0 || order[k] >= n) return 1;
    if (grad && !dL_dimg) return 1;
    if (dL_dT && !dL_dimg) return 1;
    const int fmt = cfg->fb_format;
    const int emu = cfg->emulate;
    const int per_frag = emu && cfg->fb_round == 1;

    /* per crop row: candidate order positions (all of them without the prefilter) */
    int32_t* rcount = (int32_t*)calloc((size_t)ch + 1, sizeof(int32_t));
    range_t* rng = (range_t*)malloc(sizeof(range_t) * (size_t)(n_order > 0 ? n_order : 1));
    /* compact gradient slot per order position */
    int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_order > 0 ? n_order : 1));
    int32_t nslot = 0;
    for (int32_t k = 0; k < n_order; ++k) {
        int32_t i = order[k];
        if (cfg->prefilter) {
            splat_range(cfg, means2d + 2 * i, conics + 3 * i, opac[i], &rng[k]);
        } else {
            rng[k].any = 1; rng[k].x0 = INT32_MIN / 2; rng[k].x1 = INT32_MAX / 2;
            rng[k].y0 = INT32_MIN / 2; rng[k].y1 = INT32_MAX / 2;
        }
        int32_t lo = rng[k].y0 - y0, hi = rng[k].y1 - y0;
        if (lo < 0) lo = 0;
        if (hi > ch - 1) hi = ch - 1;
        int32_t xl = rng[k].x0, xh = rng[k].x1;
        int in_x = !(xh < x0 || xl > x0 + cw - 1);
        if (!rng[k].any || lo > hi || !in_x) { rng[k].any = 0; slot[k] = -1; continue; }
        slot[k] = nslot++;
        for (int32_t r = lo; r <= hi; ++r) rcount[r + 1]++;
    }
    for (int32_t r = 0; r < ch; ++r) rcount[r + 1] += rcount[r];
    int64_t total = rcount[ch];
    int32_t* rlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int32_t* fillp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ch > 0 ? ch : 1));
    for (int32_t r = 0; r < ch; ++r) fillp[r] = rcount[r];
    for (int32_t k = 0; k < n_order; ++k) {
        if (!rng[k].any) continue;
        int32_t lo = rng[k].y0 - y0, hi = rng[k].y1 - y0;
        if (lo < 0) lo = 0;
        if (hi > ch - 1) hi = ch - 1;
        for (int32_t r = lo; r <= hi; ++r) rlist[fillp[r]++] = k;   /* keeps the depth order */
    }
    free(fillp);

    int nth = cfg->nthreads > 0 ? cfg->nthreads : 1;
#ifdef _OPENMP
    if (nth > omp_get_max_threads()) nth = omp_get_max_threads();
#else
    nth = 1;
#endif
    double* gbuf = NULL;
    if (grad) gbuf = (double*)calloc((size_t)nth * (size_t)(nslot > 0 ? nslot : 1) * 9, sizeof(double));

    const double amin = cfg->alpha_min, amax = cfg->alpha_max;
    const double tf = cfg->t_min_fwd, tb = cfg->t_min_bwd;
    const int64_t npix = (int64_t)cw * ch;
    const double* bg = cfg->background;
    double* gbg = (double*)calloc((size_t)nth * 3, sizeof(double));

#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
    for (int64_t pix = 0; pix < npix; ++pix) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int32_t ly = (int32_t)(pix / cw), lx = (int32_t)(pix % cw);
        int32_t X = x0 + lx, Y = y0 + ly;
        double px = X + 0.5, py = Y + 0.5;
        const int32_t* cand = rlist + rcount[ly];
        int32_t ncand = rcount[ly + 1] - rcount[ly];
        int32_t amb = 0, cov = 0, live = 0;

        /* forward: Eq. 2 with the Eq. 5 transmittance recurrence */
        double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
        for (int32_t j = 0; j < ncand; ++j) {
            int32_t k = cand[j];
            if (X < rng[k].x0 || X > rng[k].x1) continue;
            int32_t i = order[k];
            frag_t f;
            eval_fragment(cfg, px, py, means2d + 2 * i, conics + 3 * i, opac[i], &f);
            amb += f.amb;
            if (f.alpha < amin) continue;
            if (tf > 0.0) {
                if (fabs(T / tf - 1.0) <= cfg->tau) amb++;
                if (T < tf) break;             /* T only decreases: every later fragment is culled */
            }
            cov++;
            for (int ch3 = 0; ch3 < 3; ++ch3) {
                double cc = rgb[3 * i + ch3];
                if (cfg->saturate && cc > 1.0) cc = 1.0;
                C[ch3] += T * f.alpha * cc;
            }
            T *= (1.0 - f.alpha);
            if (per_frag) {
                for (int ch3 = 0; ch3 < 3; ++ch3) C[ch3] = oracle_round_fmt(C[ch3], fmt);
                T = oracle_round_fmt(T, fmt);
            }
        }
        /* the background shows through the final transmittance; T stays the splats' product */
        for (int ch3 = 0; ch3 < 3; ++ch3) C[ch3] += T * bg[ch3];
        if (per_frag)
            for (int ch3 = 0; ch3 < 3; ++ch3) C[ch3] = oracle_round_fmt(C[ch3], fmt);
        if (emu) {      /* the state written back to the framebuffer */
            for (int ch3 = 0; ch3 < 3; ++ch3) C[ch3] = oracle_round_fmt(C[ch3], fmt);
            T = oracle_round_fmt(T, fmt);
        }
        if (out_img)
            for (int ch3 = 0; ch3 < 3; ++ch3) out_img[(int64_t)ch3 * npix + pix] = C[ch3];
        if (out_T) out_T[pix] = T;
        if (out_cov) out_cov[pix] = cov;

        /* backward: Procedure 1 (ComputeGradient), front to back from (C'_1, T_1) = (C, 1) */
        if (dL_dimg) {
            double G[3];
            for (int ch3 = 0; ch3 < 3; ++ch3)
                G[ch3] = dL_dimg[(int64_t)ch3 * W * H + (int64_t)Y * W + X];
            /* dL/dT_final: T_final = prod_j (1 - alpha_j), so it adds -dL/dT T_final / (1 - alpha_i)
               to dL/dalpha_i; and dL/dbg = dL/dC T_final */
            const double gTT = dL_dT ? dL_dT[(int64_t)Y * W + X] * T : 0.0;
            for (int ch3 = 0; ch3 < 3; ++ch3) gbg[(size_t)tid * 3 + ch3] += G[ch3] * T;
            double Cp[3] = {C[0], C[1], C[2]}, Tb = 1.0;
            double* gb = gbuf ? gbuf + (size_t)tid * (size_t)nslot * 9 : NULL;
            for (int32_t j = 0; j < ncand; ++j) {
                int32_t k = cand[j];
                if (X < rng[k].x0 || X > rng[k].x1) continue;
                int32_t i = order[k];
                frag_t f;
                eval_fragment(cfg, px, py, means2d + 2 * i, conics + 3 * i, opac[i], &f);
                if (f.alpha < amin) continue;            /* cullingFlag: splat boundary */
                if (fabs(Tb / tb - 1.0) <= cfg->tau) amb++;
                if (Tb < tb) break;                      /* cullingFlag: T-culling; state frozen */
                live++;
                double cc[3];
                int sat[3];
                for (int ch3 = 0; ch3 < 3; ++ch3) {
                    cc[ch3] = rgb[3 * i + ch3];
                    sat[ch3] = cfg->saturate && cc[ch3] > 1.0;
                    if (sat[ch3]) cc[ch3] = 1.0;
                }
                double dL_dc[3], dL_dalpha = 0.0;
                for (int ch3 = 0; ch3 < 3; ++ch3) {
                    dL_dc[ch3] = sat[ch3] ? 0.0 : G[ch3] * f.alpha * Tb;               /* Eq. 3 */
                    dL_dalpha += G[ch3] * (cc[ch3] * Tb - Cp[ch3]);                      /* Eq. 7 */
                }
                dL_dalpha = (dL_dalpha - gTT) / (1.0 - f.alpha);
                for (int ch3 = 0; ch3 < 3; ++ch3) Cp[ch3] -= Tb * f.alpha * cc[ch3];  /* Eq. 6 */
                Tb *= (1.0 - f.alpha);                                                  /* Eq. 5 */
                if (per_frag) {
                    for (int ch3 = 0; ch3 < 3; ++ch3) Cp[ch3] = oracle_round_fmt(Cp[ch3], fmt);
                    Tb = oracle_round_fmt(Tb, fmt);
                }
                if (gb) {
                    double* g = gb + (size_t)slot[k] * 9;
                    double a = conics[3 * i], b = conics[3 * i + 1], c = conics[3 * i + 2];
                    if (fabs(f.araw / amax - 1.0) <= cfg->beta) amb++;
                    if (f.araw < amax) {            /* alpha not clamped */
                        double dL_do = dL_dalpha * f.e;
                        double dL_dq = dL_dalpha * (-0.5 * f.araw);
                        g[0] += dL_dq * (-2.0) * (a * f.dx + b * f.dy);   /* mean x */
                        g[1] += dL_dq * (-2.0) * (b * f.dx + c * f.dy);   /* mean y */
                        g[2] += dL_dq * f.dx * f.dx;                      /* conic a */
                        g[3] += dL_dq * 2.0 * f.dx * f.dy;                /* conic b */
                        g[4] += dL_dq * f.dy * f.dy;                      /* conic c */
                        g[5] += dL_do;                                    /* opacity */
                    }
                    g[6] += dL_dc[0];
                    g[7] += dL_dc[1];
                    g[8] += dL_dc[2];
                }
            }
        }
        if (out_live) out_live[pix] = live;
        if (out_amb) out_amb[pix] = amb;
    }

    if (grad_bg) {
        grad_bg[0] = grad_bg[1] = grad_bg[2] = 0.0;
        for (int t = 0; t < nth; ++t)
            for (int ch3 = 0; ch3 < 3; ++ch3) grad_bg[ch3] += gbg[(size_t)t * 3 + ch3];
    }
    free(gbg);
    if (grad) {
        memset(grad, 0, sizeof(double) * (size_t)n * 9);
        for (int32_t k = 0; k < n_order; ++k) {
            if (slot[k] < 0) continue;
            int32_t i = order[k];
            for (int t = 0; t < nth; ++t) {
                const double* g = gbuf + ((size_t)t * nslot + slot[k]) * 9;
                for (int j = 0; j < 9; ++j) grad[(size_t)i * 9 + j] += g[j];
            }
        }
    }
    free(gbuf);
    free(rlist);
    free(rcount);
    free(rng);
    free(slot);
    return 0;
}

/*
 * Per-fragment trace of one pixel (pure FP64 unless cfg->emulate), for tests of the
 * recurrences: for each fragment with alpha >= alpha_min in order, writes
 * [order position, alpha, T_i, C'_i (3), dL/dalpha_i, live] (8 doubles). Returns the count.
 * `C_final` receives the forward colour used as C'_1.
 */
int32_t oracle_pixel_trace(const ocfg_t* cfg, int32_t n, const double* means2d,
                           const double* conics, const double* opac, const double* rgb,
                           const int32_t* order, int32_t n_order, double px, double py,
                           const double* G, int32_t max_frag, double* out, double* C_final)
{
    (void)n;
    const int fmt = cfg->fb_format;
    const int per_frag = cfg->emulate && cfg->fb_round == 1;
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    for (int32_t k = 0; k < n_order; ++k) {
        int32_t i = order[k];
        frag_t f;
        eval_fragment(cfg, px, py, means2d + 2 * i, conics + 3 * i, opac[i], &f);
        if (f.alpha < cfg->alpha_min) continue;
        if (cfg->t_min_fwd > 0.0 && T < cfg->t_min_fwd) break;
        for (int c3 = 0; c3 < 3; ++c3) {
            double cc = rgb[3 * i + c3];
            if (cfg->saturate && cc > 1.0) cc = 1.0;
            C[c3] += T * f.alpha * cc;
        }
        T *= 1.0 - f.alpha;
        if (per_frag) {
            for (int c3 = 0; c3 < 3; ++c3) C[c3] = oracle_round_fmt(C[c3], fmt);
            T = oracle_round_fmt(T, fmt);
        }
    }
    for (int c3 = 0; c3 < 3; ++c3) C[c3] += T * cfg->background[c3];
    if (cfg->emulate)
        for (int c3 = 0; c3 < 3; ++c3) C[c3] = oracle_round_fmt(C[c3], fmt);
    for (int c3 = 0; c3 < 3; ++c3) C_final[c3] = C[c3];
    double Cp[3] = {C[0], C[1], C[2]}, Tb = 1.0;
    int32_t cnt = 0;
    int frozen = 0;
    for (int32_t k = 0; k < n_order && cnt < max_frag; ++k) {
        int32_t i = order[k];
        frag_t f;
        eval_fragment(cfg, px, py, means2d + 2 * i, conics + 3 * i, opac[i], &f);
        if (f.alpha < cfg->alpha_min) continue;
        double* o = out + (size_t)cnt * 8;
        o[0] = k; o[1] = f.alpha; o[2] = Tb; o[3] = Cp[0]; o[4] = Cp[1]; o[5] = Cp[2];
        if (frozen || Tb < cfg->t_min_bwd) {
            frozen = 1;
            o[6] = 0.0; o[7] = 0.0;
        } else {
            double cc[3], ga = 0.0;
            for (int c3 = 0; c3 < 3; ++c3) {
                cc[c3] = rgb[3 * i + c3];
                if (cfg->saturate && cc[c3] > 1.0) cc[c3] = 1.0;
                ga += G[c3] * (cc[c3] * Tb - Cp[c3]);
            }
            o[6] = ga / (1.0 - f.alpha);
            o[7] = 1.0;
            for (int c3 = 0; c3 < 3; ++c3) Cp[c3] -= Tb * f.alpha * cc[c3];
            Tb *= 1.0 - f.alpha;
            if (per_frag) {
                for (int c3 = 0; c3 < 3; ++c3) Cp[c3] = oracle_round_fmt(Cp[c3], fmt);
                Tb = oracle_round_fmt(Tb, fmt);
            }
        }
        cnt++;
    }
    return cnt;
}

int32_t oracle_version(void) { return 1; }
