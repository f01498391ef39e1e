/* Plain FP64 line integrals of a cosine-weighted projection (test
 * infrastructure; the CPU oracle's only compiled part).
 *
 * G(alpha_m, t_k) = ds * sum_{j=0}^{n_s-1} bilinear(img; u0 + t cos a - s_j sin a,
 *                                                    v0 + t sin a + s_j cos a),
 * alpha_m = m * dalpha, t_k = -t_max + k * dt, s_j = (j - (n_s - 1) / 2) * ds.
 * Bilinear interpolation at pixel centres (column i at u = i, row j at v = j);
 * neighbours outside the image contribute zero.  Every sample is summed,
 * including those that fall outside the image.
 *
 * This is the integral along a detector line that Grangeat's intermediate
 * function (Eq. 1) differentiates; the weighting and the derivative are done
 * by the Python caller.
 */
#include <math.h>

static double pixel(const double *img, int W, int H, int i, int j)
{
    if (i < 0 || j < 0 || i >= W || j >= H)
        return 0.0;
    return img[(long)j * W + i];
}

static double bilinear(const double *img, int W, int H, double x, double y)
{
    double fx0 = floor(x), fy0 = floor(y);
    int i0 = (int)fx0, j0 = (int)fy0;
    double fx = x - fx0, fy = y - fy0;
    double top = (1.0 - fx) * pixel(img, W, H, i0, j0) + fx * pixel(img, W, H, i0 + 1, j0);
    double bot = (1.0 - fx) * pixel(img, W, H, i0, j0 + 1) + fx * pixel(img, W, H, i0 + 1, j0 + 1);
    return (1.0 - fy) * top + fy * bot;
}

void oracle_line_integrals(const double *img, int W, int H, double u0, double v0,
                           double dalpha, double t_max, double dt, double ds, int n_s,
                           const int *m, const int *k, long n_cells, double *out)
{
    for (long c = 0; c < n_cells; ++c) {
        double alpha = m[c] * dalpha;
        double t = -t_max + k[c] * dt;
        double ca = cos(alpha), sa = sin(alpha);
        double acc = 0.0;
        for (int j = 0; j < n_s; ++j) {
            double s = (j - 0.5 * (n_s - 1)) * ds;
            double x = u0 + t * ca - s * sa;
            double y = v0 + t * sa + s * ca;
            acc += bilinear(img, W, H, x, y);
        }
        out[c] = ds * acc;
    }
}
