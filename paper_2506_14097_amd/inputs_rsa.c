/* inputs_rsa.c -- random sequential addition of non-overlapping spheres in a
 * periodic box (input generation only; no part of the time-step).
 *
 * Spheres are placed in the order given; each gets up to max_attempts uniform
 * random positions (splitmix64 stream from `seed`) and keeps the first that
 * clears every placed sphere (periodic minimum image).  A uniform cell grid
 * of edge >= 2 r_max limits the checks to the 27 (9 planar) neighbour cells.
 * Returns the number of spheres placed (n on success). */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double unif(uint64_t *s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

int rsa_spheres(int n, const double *radii, const int *order, const double box[3], int planar, uint64_t seed,
                int max_attempts, double *pos /* 3n */) {
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) rmax = radii[i] > rmax ? radii[i] : rmax;
    int dims = planar ? 2 : 3;
    int nc[3] = {1, 1, 1};
    double cs[3] = {1, 1, 1};
    for (int k = 0; k < dims; ++k) {
        nc[k] = (int)floor(box[k] / (2.0 * rmax));
        if (nc[k] < 1) nc[k] = 1;
        cs[k] = box[k] / nc[k];
    }
    long long ncell = (long long)nc[0] * nc[1] * nc[2];
    int *head = malloc(sizeof(int) * ncell), *next = malloc(sizeof(int) * (n + 1));
    for (long long c = 0; c < ncell; ++c) head[c] = -1;
    uint64_t st = seed;
    int placed = 0;
    for (int t = 0; t < n; ++t) {
        int i = order[t];
        double r = radii[i];
        int ok = 0;
        for (int att = 0; att < max_attempts && !ok; ++att) {
            double p[3] = {0, 0, 0};
            int c[3] = {0, 0, 0};
            for (int k = 0; k < dims; ++k) {
                p[k] = unif(&st) * box[k];
                c[k] = (int)(p[k] / cs[k]);
                if (c[k] >= nc[k]) c[k] = nc[k] - 1;
            }
            ok = 1;
            int lo2 = planar ? 0 : -1, hi2 = planar ? 0 : 1;
            for (int dz = lo2; dz <= hi2 && ok; ++dz)
                for (int dy = -1; dy <= 1 && ok; ++dy)
                    for (int dx = -1; dx <= 1 && ok; ++dx) {
                        int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                        int d3[3] = {dx, dy, dz};
                        int dup = 0;
                        for (int k = 0; k < 3; ++k) {
                            cc[k] = ((cc[k] % nc[k]) + nc[k]) % nc[k];
                            /* with 1 or 2 cells in a direction, skip offsets that
                             * revisit a cell already scanned */
                            if (nc[k] == 1 && d3[k] != 0) dup = 1;
                            if (nc[k] == 2 && d3[k] == 1) dup = 1;
                        }
                        if (dup) continue;
                        long long id = ((long long)cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                        for (int j = head[id]; j >= 0; j = next[j]) {
                            double d2 = 0.0;
                            for (int k = 0; k < dims; ++k) {
                                double d = pos[3 * j + k] - p[k];
                                d -= box[k] * nearbyint(d / box[k]);
                                d2 += d * d;
                            }
                            double rr = r + radii[j];
                            if (d2 < rr * rr) { ok = 0; break; }
                        }
                    }
            if (ok) {
                for (int k = 0; k < 3; ++k) pos[3 * i + k] = p[k];
                long long id = ((long long)c[2] * nc[1] + c[1]) * nc[0] + c[0];
                next[i] = head[id];
                head[id] = i;
                ++placed;
            }
        }
        if (!ok) break;
    }
    free(head);
    free(next);
    return placed;
}
