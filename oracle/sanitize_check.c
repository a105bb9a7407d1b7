/*
 * Memory- and UB-safety driver for the CPU oracle (test infrastructure only).
 *
 * It compiles gs_oracle.c into one executable with this file, so that the tests can
 * build it with AddressSanitizer and UndefinedBehaviorSanitizer on the host and run
 * every exported oracle routine over small seeded scenes that reach its edge cases:
 * Gaussians behind the near plane, a zero quaternion, opacities past alpha_max, a
 * Gaussian far outside the field of view (Jacobian clamp), a view whose size is not a
 * multiple of the tile, an empty scene and an empty pixel list.  It prints one line of
 * sums of everything it computed; the tests compare that line between a sanitized and
 * a plain build (same thread count), so the sanitizers change no result.
 *
 * The scene comes from a 64-bit linear congruential generator (Knuth's MMIX constants);
 * it draws no number the method itself uses.
 */
#include "gs_oracle.c"

#include <stdio.h>

static uint64_t lcg_state;

static double urand(double lo, double hi)
{
    lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return lo + (hi - lo) * (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static double sum_array(const double *a, int64_t n)
{
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += a[k];
    return s;
}

/* Runs every oracle routine on one scene of n Gaussians; returns 0 on success. */
static int run_scene(int64_t n, int32_t width, int32_t height, int32_t tile, uint64_t seed)
{
    lcg_state = seed;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    double *means = calloc(3 * nn, sizeof(double)), *ls = calloc(3 * nn, sizeof(double));
    double *quats = calloc(4 * nn, sizeof(double)), *op = calloc(nn, sizeof(double));
    double *rgb = calloc(3 * nn, sizeof(double));
    if (!means || !ls || !quats || !op || !rgb) return 1;
    for (int64_t g = 0; g < n; ++g) {
        means[g] = urand(-1.5, 1.5);
        means[nn + g] = urand(-1.0, 1.0);
        means[2 * nn + g] = urand(0.6, 4.0);
        for (int d = 0; d < 3; ++d) ls[d * nn + g] = urand(-3.0, -1.2);
        for (int d = 0; d < 4; ++d) quats[d * nn + g] = urand(-1.0, 1.0);
        op[g] = urand(-3.0, 6.0);
        for (int d = 0; d < 3; ++d) rgb[d * nn + g] = urand(0.0, 1.0);
    }
    if (n > 4) {
        means[2 * nn + 0] = -1.0;                   /* behind the camera */
        means[2 * nn + 1] = 0.1;                    /* in front of the near plane */
        for (int d = 0; d < 4; ++d) quats[d * nn + 2] = 0.0; /* zero quaternion */
        op[3] = 9.0;                                /* alpha past alpha_max */
        means[4] = 3.0;                             /* far off axis: Jacobian clamp */
        means[2 * nn + 4] = 1.0;
        for (int d = 0; d < 3; ++d) ls[d * nn + 4] = 0.0;
    }
    orc_gaussians G = {n, means, ls, quats, op, rgb};
    orc_view V = {width, height, 0.9 * width, 0.9 * width, 0.5 * width, 0.5 * height,
                  {1, 0, 0, 0.05, 0, 1, 0, -0.02, 0, 0, 1, 0.1}};
    orc_settings S = {0.2, 1.0 / 255.0, 0.99, 1e-4, 0.3, 1.3, {0.1, 0.2, 0.3}, 1.0};

    orc_proj *P = calloc(nn, sizeof(orc_proj));
    const int64_t npix = (int64_t)width * height;
    int32_t *pix = malloc(sizeof(int32_t) * 2 * (size_t)(npix > 0 ? npix : 1));
    orc_pixel *px = calloc((size_t)(npix > 0 ? npix : 1), sizeof(orc_pixel));
    if (!P || !pix || !px) return 1;
    for (int32_t j = 0; j < height; ++j)
        for (int32_t i = 0; i < width; ++i) {
            pix[2 * ((int64_t)j * width + i)] = i;
            pix[2 * ((int64_t)j * width + i) + 1] = j;
        }
    if (orc_project(&G, &V, &S, P)) return 2;
    if (orc_render(&G, &V, &S, P, npix, pix, px)) return 3;
    if (orc_render(&G, &V, &S, P, 0, pix, px)) return 3;

    double img = 0.0;
    int64_t frags = 0, flags = 0;
    for (int64_t p = 0; p < npix; ++p) {
        img += px[p].rgb[0] + px[p].rgb[1] + px[p].rgb[2] + px[p].depth + px[p].alpha +
               px[p].pm_world[0] + px[p].pm_cam[1] + px[p].pm_eq5[2] + px[p].T_final;
        frags += px[p].n_frag;
        flags += px[p].ambiguous != 0;
    }

    /* Upstream gradients for the backward and the frozen-trace loss. */
    double *g_rgb = malloc(sizeof(double) * 3 * (size_t)(npix > 0 ? npix : 1));
    double *g_dep = malloc(sizeof(double) * (size_t)(npix > 0 ? npix : 1));
    double *g_alp = malloc(sizeof(double) * (size_t)(npix > 0 ? npix : 1));
    double *g_pm = malloc(sizeof(double) * 3 * (size_t)(npix > 0 ? npix : 1));
    if (!g_rgb || !g_dep || !g_alp || !g_pm) return 1;
    for (int64_t p = 0; p < npix; ++p) {
        for (int d = 0; d < 3; ++d) g_rgb[3 * p + d] = urand(-1.0, 1.0);
        g_dep[p] = urand(-1.0, 1.0);
        g_alp[p] = urand(-1.0, 1.0);
        for (int d = 0; d < 3; ++d) g_pm[3 * p + d] = urand(-1.0, 1.0);
    }

    double *gbuf = calloc(15 * nn + 6, sizeof(double));
    if (!gbuf) return 1;
    double grad_sum = 0.0;
    for (int32_t frame = 0; frame < 3; ++frame) {
        memset(gbuf, 0, sizeof(double) * (15 * nn + 6));
        orc_grads R = {gbuf, gbuf + 3 * nn, gbuf + 6 * nn, gbuf + 10 * nn, gbuf + 11 * nn,
                       gbuf + 14 * nn};
        if (orc_backward(&G, &V, &S, P, frame, npix, pix, g_rgb, g_dep, g_alp, g_pm, &R)) return 4;
        grad_sum += sum_array(gbuf, (int64_t)(15 * nn + 6));
    }

    /* Frozen trace and its loss. */
    int64_t *offs = malloc(sizeof(int64_t) * (size_t)(npix + 1));
    if (!offs) return 1;
    const int64_t need = orc_trace(&G, &V, &S, P, npix, pix, 0, offs, NULL, NULL);
    const int64_t cap = need < 0 ? -need : need;
    int64_t *fg = malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
    int8_t *fc = malloc((size_t)(cap > 0 ? cap : 1));
    int8_t *cxy = malloc(2 * nn);
    if (!fg || !fc || !cxy) return 1;
    if (orc_trace(&G, &V, &S, P, npix, pix, cap, offs, fg, fc) != cap) return 5;
    for (int64_t g = 0; g < n; ++g) {
        cxy[2 * g] = (int8_t)P[g].clamp_x;
        cxy[2 * g + 1] = (int8_t)P[g].clamp_y;
    }
    const double loss = orc_replay_loss(&G, &V, &S, cxy, 2, npix, pix, offs, fg, fc, g_rgb,
                                        g_dep, g_alp, g_pm);
    if (loss != loss) return 6;

    /* Tile lists. */
    const int64_t tneed = orc_tile_sets(P, n, width, height, tile, S.alpha_min, 0, NULL, NULL, NULL);
    const int64_t tcap = tneed < 0 ? -tneed : tneed;
    int32_t *tt = malloc(sizeof(int32_t) * (size_t)(tcap > 0 ? tcap : 1));
    int64_t *tg = malloc(sizeof(int64_t) * (size_t)(tcap > 0 ? tcap : 1));
    double *tr = malloc(sizeof(double) * (size_t)(tcap > 0 ? tcap : 1));
    if (!tt || !tg || !tr) return 1;
    if (orc_tile_sets(P, n, width, height, tile, S.alpha_min, tcap, tt, tg, tr) != tcap) return 7;
    int64_t exact = 0;
    for (int64_t k = 0; k < tcap; ++k) exact += tr[k] <= 1.0;

    /* SE(3) exponential with both parts non-zero and at zero rotation. */
    double T[12];
    const double xi1[6] = {0.1, -0.2, 0.3, 0.4, -0.1, 0.2}, xi0[6] = {0.1, 0.2, 0.3, 0, 0, 0};
    orc_se3_exp_left(xi1, V.T, T);
    double se3 = sum_array(T, 12);
    orc_se3_exp_left(xi0, V.T, T);
    se3 += sum_array(T, 12);

    printf("n=%lld %dx%d B=%d img=%.17g frags=%lld flags=%lld grad=%.17g loss=%.17g pairs=%lld "
           "exact=%lld se3=%.17g\n",
           (long long)n, width, height, tile, img, (long long)frags, (long long)flags, grad_sum,
           loss, (long long)tcap, (long long)exact, se3);

    free(means); free(ls); free(quats); free(op); free(rgb); free(P); free(pix); free(px);
    free(g_rgb); free(g_dep); free(g_alp); free(g_pm); free(gbuf); free(offs); free(fg);
    free(fc); free(cxy); free(tt); free(tg); free(tr);
    return 0;
}

int main(int argc, char **argv)
{
    orc_set_num_threads(argc > 1 ? atoi(argv[1]) : 2);
    int rc = run_scene(96, 37, 29, 16, 12345u);
    if (!rc) rc = run_scene(48, 64, 48, 8, 777u);
    if (!rc) rc = run_scene(0, 20, 10, 16, 1u);
    if (!rc) rc = run_scene(8, 1, 1, 16, 99u);
    if (rc) fprintf(stderr, "oracle routine failed: code %d\n", rc);
    return rc;
}
