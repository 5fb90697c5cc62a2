/* Host sanitizer run of the CPU oracle (test infrastructure): every oracle
 * entry point on small random inputs of awkward sizes, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by test_sanitizers.py.
 * Exits non-zero on the first oracle error; the sanitizers abort on their
 * own findings. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_census(const uint8_t *img, int W, int H, int pitch, int n, uint64_t *out);
int oracle_cost(const uint64_t *cl, const uint64_t *cr, int W, int H, int n, int w, const int32_t *d_lo,
                uint8_t *out);
int oracle_path(const uint8_t *cost, int W, int H, int w, int du, int dv, int p1, int p2, uint16_t *out);
int oracle_sum(const uint8_t *cost, int W, int H, int w, int npaths, int p1, int p2, uint32_t *out);
int oracle_wta(const uint32_t *S, int W, int H, int w, const int32_t *d_lo, uint16_t *dint, float *dsub);
int oracle_sgm(const uint8_t *left, const uint8_t *right, int W, int H, int pitch, int n, int w, int npaths,
               int p1, int p2, const int32_t *d_lo, uint16_t *dint, float *dsub);
int oracle_window_from_road(double a0, double a1, double phi, int W, int H, int w, int mode, double delta,
                            int32_t *d_lo);
int oracle_sgm_win(const uint8_t *left, const uint8_t *right, int W, int H, int pitch, int n, int w,
                   int npaths, int p1, int p2, const int32_t *lo, uint16_t *dint, float *dsub);
int oracle_downsample4(const uint8_t *img, int W, int H, int pitch, uint8_t *out);

static uint32_t rng_state = 12345u;
static uint32_t rnd(void)
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

#define CHECK(x)                                                   \
    do {                                                           \
        if ((x) != 0) {                                            \
            fprintf(stderr, "oracle call failed: %s\n", #x);       \
            return 1;                                              \
        }                                                          \
    } while (0)

static int one(int W, int H, int n, int w, int npaths)
{
    const int pitch = W + 3;
    uint8_t *L = malloc((size_t)pitch * H), *R = malloc((size_t)pitch * H);
    uint64_t *cl = malloc(sizeof(uint64_t) * W * H), *cr = malloc(sizeof(uint64_t) * W * H);
    uint8_t *C = malloc((size_t)W * H * w);
    uint16_t *Lr = malloc(sizeof(uint16_t) * W * H * w), *dint = malloc(sizeof(uint16_t) * W * H);
    uint32_t *S = malloc(sizeof(uint32_t) * W * H * w);
    float *dsub = malloc(sizeof(float) * W * H);
    int32_t *dlo = malloc(sizeof(int32_t) * H), *lo = malloc(sizeof(int32_t) * W * H);
    uint8_t *small = malloc((size_t)(W / 4 + 1) * (H / 4 + 1));
    for (int i = 0; i < pitch * H; ++i) {
        L[i] = (uint8_t)rnd();
        R[i] = (uint8_t)rnd();
    }
    for (int v = 0; v < H; ++v) dlo[v] = (int32_t)(rnd() % 5);
    for (int i = 0; i < W * H; ++i) lo[i] = (int32_t)(rnd() % 9);
    CHECK(oracle_census(L, W, H, pitch, n, cl));
    CHECK(oracle_census(R, W, H, pitch, n, cr));
    CHECK(oracle_cost(cl, cr, W, H, n, w, dlo, C));
    for (int r = 0; r < 8; ++r) {
        static const int du[8] = {1, -1, 0, 0, 1, -1, 1, -1}, dv[8] = {0, 0, 1, -1, 1, 1, -1, -1};
        CHECK(oracle_path(C, W, H, w, du[r], dv[r], 10, 120, Lr));
    }
    CHECK(oracle_sum(C, W, H, w, npaths, 10, 120, S));
    CHECK(oracle_wta(S, W, H, w, dlo, dint, dsub));
    CHECK(oracle_sgm(L, R, W, H, pitch, n, w, npaths, 10, 120, dlo, dint, dsub));
    if (w <= 16) CHECK(oracle_sgm_win(L, R, W, H, pitch, n, w, npaths, 10, 120, lo, dint, dsub));
    if (W >= 4 && H >= 4) CHECK(oracle_downsample4(L, W, H, pitch, small));
    CHECK(oracle_window_from_road(20.0, 0.1, 0.03, W, H, w, 0, 0.0, dlo));
    CHECK(oracle_window_from_road(20.0, 0.1, 0.03, W, H, w, 1, 1.5, dlo));
    free(L); free(R); free(cl); free(cr); free(C); free(Lr); free(dint); free(S); free(dsub); free(dlo);
    free(lo); free(small);
    return 0;
}

int main(void)
{
    static const int cases[][5] = {{1, 1, 3, 1, 4},   {2, 9, 5, 16, 8},  {13, 1, 7, 24, 8}, {17, 11, 7, 16, 8},
                                   {31, 7, 5, 64, 4}, {9, 23, 3, 128, 8}, {6, 5, 7, 256, 8}};
    for (unsigned i = 0; i < sizeof cases / sizeof cases[0]; ++i)
        if (one(cases[i][0], cases[i][1], cases[i][2], cases[i][3], cases[i][4])) return 1;
    puts("oracle sanitizer run clean");
    return 0;
}
