/*
 * FP64 brute-force spectrum compositor: the oracle for the render path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is compiled into liboracle_raster.so and
 * is called by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark. Nothing on the product path links or calls it, and it shares no
 * code, header or constant table with the HIP library.
 *
 * What it computes (paper Sec. 3.2, the front-to-back blending equation for
 * C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j), with the 2D Gaussian kernel of
 * Sec. 4.1, eq. for K(mu, Sigma, delta) = delta * exp(-d^T Sigma^-1 d / 2)):
 *
 *   for every listed pixel (x, y) [pixel units], in ascending (depth, id) order:
 *     d = (x - mx, y - my);  q = d^T Sigma^-1 d
 *     skip if q > 9                         (3-sigma cutoff, 9 itself is kept)
 *     alpha = min(0.99, opacity * exp(-q/2))
 *     skip if alpha < 1/255
 *     T' = T (1 - alpha); if T' < 1e-4 the pixel is finished and this Gaussian
 *     is NOT added; otherwise C += amp * alpha * T and T = T'.
 *
 * The thresholds are the FP32 constants 0.99f, 1.0f/255.0f and 1e-4f, widened
 * to FP64 by the caller. Every Gaussian is visited (no binning, no tiles).
 *
 * Azimuth wrap (optional, consts[4] = the grid width W in pixels, 0 = off):
 * azimuth is periodic (0 and 360 degrees are one direction), so the
 * horizontal displacement is taken to the nearest image of the mean,
 * dx = (x - mx) - W round((x - mx) / W).
 *
 * Decision ambiguity. FP32 and FP64 can disagree on a discrete decision whose
 * FP64 quantity lies very close to its threshold. Each such decision (q vs 9,
 * alpha vs 1/255, T' vs 1e-4, within a relative margin) is "flagged", and the
 * walk is forked: the other branch is followed too. The caller receives every
 * reachable result (up to ORACLE_MAX_LEAVES); a GPU value is acceptable if it
 * matches any of them. When the fork budget runs out, the remaining flagged
 * decisions are not forked and a sound extra tolerance ("bound") is returned.
 *
 * The gradient entry point holds every decision at its FP64 outcome and
 * differentiates the composited value exactly (Sec. 3.2 blending rule):
 *   dC/damp_i   = alpha_i T_i
 *   dC/dalpha_i = amp_i T_i - (sum_{j>i} amp_j alpha_j T_j) / (1 - alpha_i)
 *   alpha_i = opacity_i exp(-q_i/2)   (zero derivative where the 0.99 clamp holds)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_LEAVES 64

typedef struct {
    int64_t n;
    const double *mx, *my;          /* mean, pixel units                      */
    const double *ixx, *ixy, *iyy;  /* inverse covariance entries             */
    const double *op, *amp;         /* opacity in (0,1), amplitude            */
    const int8_t *live;             /* 0: culled (non-finite or det <= 0)    */
    const int64_t *order;           /* ascending (depth, id)                  */
    double amax, amin, tmin, qmax;  /* 0.99f, 1/255.f, 1e-4f, 9               */
    double period;                  /* azimuth period W (0: no wrap)          */
    double mq, ma, mt;              /* relative flag margins                  */
    double ampmax;                  /* max |amp| over live Gaussians          */
} scene_t;

typedef struct {
    double vals[ORACLE_MAX_LEAVES];
    int n;
    int overflow;  /* number of flagged decisions that were not forked */
    double bound;  /* extra tolerance covering the unforked decisions  */
} leaves_t;

/* Horizontal displacement of pixel column px from a mean: with a period
 * (azimuth wrap) the nearest image of the mean. */
static double disp_x(double px, double mx, double period)
{
    const double d = px - mx;
    return period > 0.0 ? d - period * nearbyint(d / period) : d;
}

static int near_threshold(double v, double thr, double rel)
{
    return fabs(v - thr) <= rel * fabs(thr);
}

/* Walk order[k0..] for one pixel from state (T, C). For the Gaussian at k0
 * only, the first `nfix` of its three decisions are fixed to fix[0..nfix-1]
 * (0 = q test, 1 = alpha test, 2 = termination test); they are neither
 * re-evaluated nor flagged. Returns the final C of this path; every path's
 * final C is appended to L. `depth` counts the active walks above this one. */
static double walk(const scene_t *s, double px, double py, int64_t k0, int nfix, const int fix[3],
                   double T, double C, int depth, int *nflags, leaves_t *L)
{
    for (int64_t k = k0; k < s->n; ++k) {
        const int64_t g = s->order[k];
        if (!s->live[g]) continue;
        const int nf = (k == k0) ? nfix : 0;
        const double dx = disp_x(px, s->mx[g], s->period), dy = py - s->my[g];
        const double q = s->ixx[g] * dx * dx + 2.0 * s->ixy[g] * dx * dy + s->iyy[g] * dy * dy;

        /* decision 0: inside the 3-sigma ellipse */
        int in = (q <= s->qmax);
        if (nf > 0) {
            in = fix[0];
        } else if (near_threshold(q, s->qmax, s->mq)) {
            ++*nflags;
            if (L->n + depth + 2 <= ORACLE_MAX_LEAVES) {
                int f[3] = {!in, 0, 0};
                int dummy = 0;
                walk(s, px, py, k, 1, f, T, C, depth + 1, &dummy, L);
            } else {
                ++L->overflow;
                L->bound += 2.0 * s->amax * T * s->ampmax;
            }
        }
        if (!in) continue;

        /* decision 1: alpha large enough to count */
        double a = s->op[g] * exp(-0.5 * q);
        if (a > s->amax) a = s->amax;
        int keep = (a >= s->amin);
        if (nf > 1) {
            keep = fix[1];
        } else if (near_threshold(a, s->amin, s->ma)) {
            ++*nflags;
            if (L->n + depth + 2 <= ORACLE_MAX_LEAVES) {
                int f[3] = {1, !keep, 0};
                int dummy = 0;
                walk(s, px, py, k, 2, f, T, C, depth + 1, &dummy, L);
            } else {
                ++L->overflow;
                L->bound += 2.0 * a * T * s->ampmax + 2.0 * s->amin * T * s->ampmax;
            }
        }
        if (!keep) continue;

        /* decision 2: transmittance would fall below the floor */
        const double Tn = T * (1.0 - a);
        int stop = (Tn < s->tmin);
        if (nf > 2) {
            stop = fix[2];
        } else if (near_threshold(Tn, s->tmin, s->mt)) {
            ++*nflags;
            if (L->n + depth + 2 <= ORACLE_MAX_LEAVES) {
                int f[3] = {1, 1, !stop};
                int dummy = 0;
                walk(s, px, py, k, 3, f, T, C, depth + 1, &dummy, L);
            } else {
                ++L->overflow;
                L->bound += T * s->ampmax;
            }
        }
        if (stop) break;
        C += s->amp[g] * a * T;
        T = Tn;
    }
    if (L->n < ORACLE_MAX_LEAVES) L->vals[L->n++] = C;
    return C;
}

/* Primary path only: final T, contributor count, last contributor position in
 * `order` (-1 if none), a 64-bit signature of the decision sequence (FNV-1a over
 * contributor ids, clamp states and the stop position), and optionally the
 * minimum T seen (monotonicity is checked by asserting T never increases). */
static double primary(const scene_t *s, double px, double py, double *T_out, int64_t *ncontrib,
                      int64_t *last, uint64_t *sig, int *monotone)
{
    double T = 1.0, C = 0.0;
    uint64_t h = 1469598103934665603ull;
    int64_t nc = 0, lk = -1, stopk = -1;
    int mono = 1;
    for (int64_t k = 0; k < s->n; ++k) {
        const int64_t g = s->order[k];
        if (!s->live[g]) continue;
        const double dx = disp_x(px, s->mx[g], s->period), dy = py - s->my[g];
        const double q = s->ixx[g] * dx * dx + 2.0 * s->ixy[g] * dx * dy + s->iyy[g] * dy * dy;
        if (!(q <= s->qmax)) continue;
        double a = s->op[g] * exp(-0.5 * q);
        int clamped = 0;
        if (a > s->amax) { a = s->amax; clamped = 1; }
        if (!(a >= s->amin)) continue;
        const double Tn = T * (1.0 - a);
        if (Tn < s->tmin) { stopk = k; break; }
        C += s->amp[g] * a * T;
        if (Tn > T) mono = 0;
        T = Tn;
        ++nc;
        lk = k;
        uint64_t v = (uint64_t)g * 2u + (uint64_t)clamped;
        for (int b = 0; b < 8; ++b) { h ^= (v >> (8 * b)) & 0xffu; h *= 1099511628211ull; }
    }
    {
        uint64_t v = (uint64_t)(stopk + 1);
        for (int b = 0; b < 8; ++b) { h ^= (v >> (8 * b)) & 0xffu; h *= 1099511628211ull; }
    }
    *T_out = T;
    *ncontrib = nc;
    *last = lk;
    *sig = h;
    *monotone = mono && T <= 1.0 && T >= s->tmin;
    return C;
}

static void fill_scene(scene_t *s, int64_t n, const double *mx, const double *my, const double *ixx,
                       const double *ixy, const double *iyy, const double *op, const double *amp,
                       const int8_t *live, const int64_t *order, const double *consts, const double *margins)
{
    s->n = n; s->mx = mx; s->my = my; s->ixx = ixx; s->ixy = ixy; s->iyy = iyy;
    s->op = op; s->amp = amp; s->live = live; s->order = order;
    s->amax = consts[0]; s->amin = consts[1]; s->tmin = consts[2]; s->qmax = consts[3];
    s->period = consts[4];
    s->mq = margins ? margins[0] : 0.0;
    s->ma = margins ? margins[1] : 0.0;
    s->mt = margins ? margins[2] : 0.0;
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (live[i] && fabs(amp[i]) > m) m = fabs(amp[i]);
    s->ampmax = m;
}

/* Render the listed pixels. Outputs (per pixel p):
 *   C[p]        primary (all-FP64-decisions) value
 *   T[p]        primary final transmittance
 *   ncontrib[p] number of Gaussians added on the primary path
 *   last[p]     position in `order` of the last added Gaussian, -1 if none
 *   sig[p]      decision signature of the primary path
 *   mono[p]     1 if T stayed monotone and inside [1e-4, 1]
 *   nflags[p]   flagged decisions met on the primary path
 *   leaves[p*ORACLE_MAX_LEAVES + j], nleaves[p]: every reachable value
 *   bound[p]    extra tolerance for decisions that could not be forked
 * margins may be NULL (no flagging; leaves then hold only the primary value). */
void oracle_render(int64_t n, const double *mx, const double *my, const double *ixx, const double *ixy,
                   const double *iyy, const double *op, const double *amp, const int8_t *live,
                   const int64_t *order, const double *consts, const double *margins, int64_t npix,
                   const int32_t *pix_x, const int32_t *pix_y, double *C, double *T, int64_t *ncontrib,
                   int64_t *last, uint64_t *sig, int8_t *mono, int32_t *nflags, double *leaves,
                   int32_t *nleaves, double *bound, int32_t *overflow)
{
    scene_t s;
    fill_scene(&s, n, mx, my, ixx, ixy, iyy, op, amp, live, order, consts, margins);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
        const double px = (double)pix_x[p], py = (double)pix_y[p];
        int m = 1;
        C[p] = primary(&s, px, py, &T[p], &ncontrib[p], &last[p], &sig[p], &m);
        mono[p] = (int8_t)m;
        leaves_t L;
        L.n = 0; L.overflow = 0; L.bound = 0.0;
        int nf = 0;
        if (margins) {
            const int none[3] = {0, 0, 0};
            walk(&s, px, py, 0, 0, none, 1.0, 0.0, 0, &nf, &L);
        } else {
            L.vals[L.n++] = C[p];
        }
        nflags[p] = nf;
        nleaves[p] = L.n;
        for (int j = 0; j < L.n; ++j) leaves[p * ORACLE_MAX_LEAVES + j] = L.vals[j];
        bound[p] = L.bound;
        overflow[p] = L.overflow;
    }
}

/* Gradient of sum_p w[p] * C[p] with every decision held at its FP64 outcome.
 * grad[g*7 + c] for c = (mx, my, ixx, ixy, iyy, opacity, amp); ixy is the single
 * off-diagonal entry, so d q / d ixy = 2 dx dy. `grad` is overwritten. With
 * margins and gflag, gflag[g] = 1 marks Gaussians with a near-threshold decision
 * at some weighted pixel (writes of 1 only, so concurrent marking is benign). */
/* With grad_abs (nullable) the same loop also accumulates, per Gaussian and
 * component, the sum over pixels of |w| times the magnitude of each term: the
 * scale of a componentwise rounding-error bound. There dC/dalpha_i is taken as
 * |amp_i| T_i + S_i' / (1 - alpha_i) with S_i' the sum of |amp_j| alpha_j T_j
 * over later contributors, and every other factor by its absolute value. */
void oracle_grad(int64_t n, const double *mx, const double *my, const double *ixx, const double *ixy,
                 const double *iyy, const double *op, const double *amp, const int8_t *live,
                 const int64_t *order, const double *consts, const double *margins, int64_t npix,
                 const int32_t *pix_x, const int32_t *pix_y, const double *w, double *grad, int8_t *gflag,
                 double *grad_abs)
{
    scene_t s;
    fill_scene(&s, n, mx, my, ixx, ixy, iyy, op, amp, live, order, consts, margins);
    memset(grad, 0, sizeof(double) * (size_t)n * 7);
    if (grad_abs) memset(grad_abs, 0, sizeof(double) * (size_t)n * 7);
    if (gflag) memset(gflag, 0, (size_t)n);
#pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)n * 7, sizeof(double));
        double *acca = grad_abs ? (double *)calloc((size_t)n * 7, sizeof(double)) : NULL;
        int64_t *cg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        double *ca = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *cT = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        int8_t *cc = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            if (w[p] == 0.0) continue;
            const double px = (double)pix_x[p], py = (double)pix_y[p];
            double T = 1.0;
            int64_t m = 0;
            for (int64_t k = 0; k < s.n; ++k) {
                const int64_t g = s.order[k];
                if (!s.live[g]) continue;
                const double dx = disp_x(px, s.mx[g], s.period), dy = py - s.my[g];
                const double q = s.ixx[g] * dx * dx + 2.0 * s.ixy[g] * dx * dy + s.iyy[g] * dy * dy;
                /* a Gaussian whose cutoff or skip decision at a weighted pixel lies
                 * within the margin of its threshold is marked: its gradient may
                 * legitimately differ from an FP32 evaluation */
                if (gflag && margins && near_threshold(q, s.qmax, s.mq)) gflag[g] = 1;
                if (!(q <= s.qmax)) continue;
                double a = s.op[g] * exp(-0.5 * q);
                int clamped = 0;
                if (a > s.amax) { a = s.amax; clamped = 1; }
                if (gflag && margins && near_threshold(a, s.amin, s.ma)) gflag[g] = 1;
                if (!(a >= s.amin)) continue;
                const double Tn = T * (1.0 - a);
                if (gflag && margins && near_threshold(Tn, s.tmin, s.mt)) gflag[g] = 1;
                if (Tn < s.tmin) break;
                cg[m] = g; ca[m] = a; cT[m] = T; cc[m] = (int8_t)clamped;
                ++m;
                T = Tn;
            }
            double S = 0.0;  /* sum over later contributors of amp_j alpha_j T_j */
            double Sa = 0.0; /* the same with |amp_j| */
            const double aw = fabs(w[p]);
            for (int64_t i = m - 1; i >= 0; --i) {
                const int64_t g = cg[i];
                const double a = ca[i], Ti = cT[i];
                const double dC_damp = a * Ti;
                const double dC_da = s.amp[g] * Ti - S / (1.0 - a);
                const double dC_da_abs = fabs(s.amp[g]) * Ti + Sa / (1.0 - a);
                S += s.amp[g] * a * Ti;
                Sa += fabs(s.amp[g]) * a * Ti;
                double *G = acc + g * 7;
                double *GA = acca ? acca + g * 7 : NULL;
                G[6] += w[p] * dC_damp;
                if (GA) GA[6] += aw * dC_damp;
                if (cc[i]) continue;
                const double dx = disp_x(px, s.mx[g], s.period), dy = py - s.my[g];
                const double q = s.ixx[g] * dx * dx + 2.0 * s.ixy[g] * dx * dy + s.iyy[g] * dy * dy;
                const double Gk = exp(-0.5 * q);
                const double dC_dop = dC_da * Gk;
                const double dC_dq = dC_da * (-0.5 * s.op[g] * Gk);
                const double ux = -2.0 * (s.ixx[g] * dx + s.ixy[g] * dy), uy = -2.0 * (s.ixy[g] * dx + s.iyy[g] * dy);
                G[0] += w[p] * dC_dq * ux;
                G[1] += w[p] * dC_dq * uy;
                G[2] += w[p] * dC_dq * dx * dx;
                G[3] += w[p] * dC_dq * 2.0 * dx * dy;
                G[4] += w[p] * dC_dq * dy * dy;
                G[5] += w[p] * dC_dop;
                if (GA) {
                    const double mq = aw * dC_da_abs * 0.5 * s.op[g] * Gk;
                    GA[0] += mq * fabs(ux);
                    GA[1] += mq * fabs(uy);
                    GA[2] += mq * dx * dx;
                    GA[3] += mq * 2.0 * fabs(dx * dy);
                    GA[4] += mq * dy * dy;
                    GA[5] += aw * dC_da_abs * Gk;
                }
            }
        }
#pragma omp critical
        {
            for (int64_t i = 0; i < n * 7; ++i) grad[i] += acc[i];
            if (acca)
                for (int64_t i = 0; i < n * 7; ++i) grad_abs[i] += acca[i];
        }
        free(acc); free(acca); free(cg); free(ca); free(cT); free(cc);
    }
}

int oracle_max_leaves(void) { return ORACLE_MAX_LEAVES; }

/* Thread count of the OpenMP loops above (timing of the oracle on a given
 * number of host cores); returns the count in effect afterwards. */
int oracle_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* Composite the listed pixels with every discrete decision taken from a base
 * scene and every value from a second one (same Gaussians, same order): the
 * 3-sigma cutoff, the alpha skip, the 0.99 clamp state and the transmittance
 * stop are decided on the base parameters (q0, alpha0, T0 of the base walk),
 * while the added terms amp alpha T use the value parameters, with alpha held
 * at 0.99 wherever the base clamp was active. At equal scenes this is the
 * primary walk of oracle_render. Around the base point it is a smooth function
 * of the value parameters whose derivative is the decisions-held gradient of
 * oracle_grad, so central differences can check that gradient without
 * rejecting samples whose perturbation flips a decision somewhere. */
void oracle_render_held(int64_t n, const double *mx0, const double *my0, const double *ixx0, const double *ixy0,
                        const double *iyy0, const double *op0, const double *mx, const double *my,
                        const double *ixx, const double *ixy, const double *iyy, const double *op,
                        const double *amp, const int8_t *live, const int64_t *order, const double *consts,
                        int64_t npix, const int32_t *pix_x, const int32_t *pix_y, double *C_out)
{
    const double amax = consts[0], amin = consts[1], tmin = consts[2], qmax = consts[3], period = consts[4];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
        const double px = (double)pix_x[p], py = (double)pix_y[p];
        double T0 = 1.0, T = 1.0, C = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const int64_t g = order[k];
            if (!live[g]) continue;
            const double ex = disp_x(px, mx0[g], period), ey = py - my0[g];
            const double q0 = ixx0[g] * ex * ex + 2.0 * ixy0[g] * ex * ey + iyy0[g] * ey * ey;
            if (!(q0 <= qmax)) continue;
            double a0 = op0[g] * exp(-0.5 * q0);
            const int clamped = a0 > amax;
            if (clamped) a0 = amax;
            if (!(a0 >= amin)) continue;
            const double Tn0 = T0 * (1.0 - a0);
            if (Tn0 < tmin) break;
            T0 = Tn0;
            const double dx = disp_x(px, mx[g], period), dy = py - my[g];
            const double q = ixx[g] * dx * dx + 2.0 * ixy[g] * dx * dy + iyy[g] * dy * dy;
            const double a = clamped ? amax : op[g] * exp(-0.5 * q);
            C += amp[g] * a * T;
            T *= 1.0 - a;
        }
        C_out[p] = C;
    }
}
