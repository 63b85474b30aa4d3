/* Random sequential addition for the synthetic electrolyte inputs: accepts
 * candidates one at a time, in draw order, when no accepted point lies
 * closer than d_min under the minimum-image convention of a periodic cube.
 * A hash grid of g^3 cells (cell diagonal < d_min, so at most one accepted
 * point per cell) finds the earlier points within reach.  Input generation
 * only: no part of the Ewald method.
 *
 * The distance test is written as the vectorised NumPy version writes it
 * (d = a - b, d -= L * rint(d / L), d0*d0 + d1*d1 + d2*d2 < d_min^2), so both
 * accept the same candidates. */
#include <math.h>
#include <stdint.h>

static double min_image(double d, double L) { return d - L * rint(d / L); }

/* Processes cand[0 .. m-1] (row-major x, y, z); appends accepted points to
 * out at *count, stopping once *count == n.  occ[g^3] holds the index of the
 * accepted point in each cell, or -1.  Returns the number of candidates
 * consumed. */
int64_t rsa_accept(double L, double d_min, int64_t g, int64_t reach, const double *cand, int64_t m,
                   double *out, int64_t *count, int64_t n, int64_t *occ)
{
    const double h = L / (double)g, d2 = d_min * d_min;
    int64_t c;
    for (c = 0; c < m && *count < n; ++c) {
        const double x = cand[3 * c], y = cand[3 * c + 1], z = cand[3 * c + 2];
        int64_t cx = (int64_t)(x / h), cy = (int64_t)(y / h), cz = (int64_t)(z / h);
        if (cx > g - 1) cx = g - 1;
        if (cy > g - 1) cy = g - 1;
        if (cz > g - 1) cz = g - 1;
        int ok = 1;
        for (int64_t ox = -reach; ok && ox <= reach; ++ox)
            for (int64_t oy = -reach; ok && oy <= reach; ++oy)
                for (int64_t oz = -reach; ok && oz <= reach; ++oz) {
                    const int64_t kx = ((cx + ox) % g + g) % g, ky = ((cy + oy) % g + g) % g,
                                  kz = ((cz + oz) % g + g) % g;
                    const int64_t id = occ[(kx * g + ky) * g + kz];
                    if (id < 0) continue;
                    const double dx = min_image(x - out[3 * id], L), dy = min_image(y - out[3 * id + 1], L),
                                 dz = min_image(z - out[3 * id + 2], L);
                    if (dx * dx + dy * dy + dz * dz < d2) ok = 0;
                }
        if (!ok) continue;
        const int64_t key = (cx * g + cy) * g + cz;
        occ[key] = *count;
        out[3 * *count] = x;
        out[3 * *count + 1] = y;
        out[3 * *count + 2] = z;
        ++*count;
    }
    return c;
}
