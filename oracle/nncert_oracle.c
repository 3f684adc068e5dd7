/*
 * CPU oracle for nearest-neighbour certificates: TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU path.
 *
 * What it computes is the plain definition of a certificate (Section 2,
 * Definition 1): for a query point i, its nearest neighbour nn_i and the two
 * smallest neighbour distances d1 <= d2, found by brute force over every other
 * point.  The paper fixes no arithmetic, so this oracle fixes one:
 *
 *   squared distance  s(i,j) = ((dx*dx) + (dy*dy)) + (dz*dz),  dx = x_j - x_i,
 *   every operation an IEEE binary32 round-to-nearest-even operation, no fused
 *   multiply-add (built with -ffp-contract=off), no flush of subnormals;
 *   nn = argmin_j s(i,j) over j != i, ties to the lowest index j;
 *   s2 = the second smallest value of the multiset {s(i,j) : j != i}
 *   (equal to s1 when the minimum is shared);
 *   d1 = sqrtf(s1), d2 = sqrtf(s2), correctly rounded;
 *   fewer than two other points: the missing distances are +inf, nn = -1 when
 *   there is no other point.
 *
 * A second routine computes the nearest neighbour with binary64 distances of
 * the same binary32 coordinates, which the tests use to tell a binary32
 * near-tie from an error.
 *
 * Layout: positions are structure-of-arrays, pos[k*n + j] is coordinate k of
 * point j, k < d.  Queries are given as a list of point indices.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops below use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of the parallel loops (k < 1: leave it unchanged). */
void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

static float sqdist32(const float *pos, int64_t n, int d, int64_t i, int64_t j)
{
    float dx = pos[j] - pos[i];
    float s = dx * dx;
    for (int k = 1; k < d; ++k) {
        float dk = pos[(int64_t)k * n + j] - pos[(int64_t)k * n + i];
        float sq = dk * dk;
        s = s + sq;
    }
    return s;
}

static double sqdist64(const float *pos, int64_t n, int d, int64_t i, int64_t j)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double dk = (double)pos[(int64_t)k * n + j] - (double)pos[(int64_t)k * n + i];
        s = s + dk * dk;
    }
    return s;
}

/* Binary32 certificate of each query by brute force over all other points. */
void orc_top2_f32(const float *pos, int64_t n, int d, const int64_t *qidx, int64_t nq,
                  int32_t *nn_out, float *d1_out, float *d2_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t i = qidx[q];
        float s1 = INFINITY, s2 = INFINITY;
        int64_t nn = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            float s = sqdist32(pos, n, d, i, j);
            if (s < s1 || (s == s1 && j < nn)) {
                s2 = s1;
                s1 = s;
                nn = j;
            } else if (s < s2) {
                s2 = s;
            }
        }
        nn_out[q] = (int32_t)nn;
        d1_out[q] = sqrtf(s1);
        d2_out[q] = sqrtf(s2);
    }
}

/* Binary64 nearest neighbour (ties to the lowest index) and its squared distance. */
void orc_nn_f64(const float *pos, int64_t n, int d, const int64_t *qidx, int64_t nq,
                int32_t *nn_out, double *s_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t i = qidx[q];
        double s1 = INFINITY;
        int64_t nn = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double s = sqdist64(pos, n, d, i, j);
            if (s < s1) {
                s1 = s;
                nn = j;
            }
        }
        nn_out[q] = (int32_t)nn;
        s_out[q] = s1;
    }
}

/* Binary64 squared distance of listed pairs (a[k], b[k]). */
void orc_pair_sqdist64(const float *pos, int64_t n, int d, const int64_t *a, const int64_t *b,
                       int64_t np, double *out)
{
    for (int64_t k = 0; k < np; ++k)
        out[k] = sqdist64(pos, n, d, a[k], b[k]);
}

/* Binary32 squared distance of listed pairs, with the certificate's formula. */
void orc_pair_sqdist32(const float *pos, int64_t n, int d, const int64_t *a, const int64_t *b,
                       int64_t np, float *out)
{
    for (int64_t k = 0; k < np; ++k)
        out[k] = sqdist32(pos, n, d, a[k], b[k]);
}
