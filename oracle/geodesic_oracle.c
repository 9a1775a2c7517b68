/*
 * Plain CPU oracle for the learned reset proposal: geodesic distance on the
 * configuration-space free grid, difficulty bins, labelled start/goal pairs,
 * the plain rejection sampler and the exact check every proposal must pass.
 * TEST INFRASTRUCTURE ONLY (same rule as navsim_oracle.c, whose Philox block
 * function this file calls; it is built into the same library).
 *
 * The paper resets to free-space start/goal poses (section 2.2.3) and says
 * nothing about difficulty; everything here is this project's reading:
 *   - C-free cell: its centre passes the clearance test of the robot's
 *     circumscribed disc (the predicate of the free-cell list);
 *   - geodesic hop count h(a, b): fewest moves between C-free cells a and b
 *     along 4-neighbour steps through C-free cells; distance = h * s;
 *   - bins: nbins equal half-open intervals of [d_lo, d_hi) metres;
 *   - a pair (a, b) is valid for bin k when both cells are C-free, their
 *     centres are at least goal_min_dist apart and h(a, b) * s lies in bin k.
 * Random choices come from Philox4x32-10 with key = seed; a uniform pick of
 * one of n items from a 32-bit word w is item (w * n) >> 32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

static void orc_words(const uint32_t key[2], uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    orc_philox4x32_10(ctr, key, w);
}

static int32_t orc_pick(uint32_t w, int64_t n) { return (int32_t)(((uint64_t)w * (uint64_t)n) >> 32); }

/* Breadth-first search from cell a over C-free cells (cfree[j W + i] != 0),
 * 4-neighbour moves, first-in first-out.  out[c] = hop count of cell c, or -1
 * when c is not reached within max_hops moves.  A start that is not C-free
 * reaches nothing (out[a] = -1 too). */
void orc_bfs_field(int32_t W, int32_t H, const uint8_t *cfree, int32_t a, int32_t max_hops,
                   int32_t *out)
{
    int64_t n = (int64_t)W * H;
    for (int64_t c = 0; c < n; ++c) out[c] = -1;
    if (a < 0 || a >= n || !cfree[a]) return;
    int32_t *q = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t head = 0, tail = 0;
    out[a] = 0;
    q[tail++] = a;
    while (head < tail) {
        int32_t c = q[head++];
        if (out[c] >= max_hops) continue;
        int32_t i = c % W, j = c / W;
        int32_t nb[4] = {i > 0 ? c - 1 : -1, i + 1 < W ? c + 1 : -1, j > 0 ? c - W : -1,
                         j + 1 < H ? c + W : -1};
        for (int d = 0; d < 4; ++d) {
            int32_t m = nb[d];
            if (m >= 0 && cfree[m] && out[m] < 0) {
                out[m] = out[c] + 1;
                q[tail++] = m;
            }
        }
    }
    free(q);
}

/* Bin of a hop count: k with d_lo + k w <= h s < d_lo + (k + 1) w, where
 * w = (d_hi - d_lo) / nbins; -1 when h < 0 or outside [d_lo, d_hi). */
int32_t orc_bin_of(double s, int32_t hops, double d_lo, double d_hi, int32_t nbins)
{
    if (hops < 0) return -1;
    double d = (double)hops * s;
    double w = (d_hi - d_lo) / (double)nbins;
    for (int32_t k = 0; k < nbins; ++k) {
        double lo = d_lo + (double)k * w, hi = d_lo + (double)(k + 1) * w;
        if (d >= lo && d < hi) return k;
    }
    return -1;
}

/* Largest hop count that falls in any bin (search depth). */
int32_t orc_max_hops(double s, double d_lo, double d_hi, int32_t nbins)
{
    int32_t h = (int32_t)(d_hi / s) + 2;
    while (h > 0 && orc_bin_of(s, h, d_lo, d_hi, nbins) < 0) --h;
    return h;
}

double orc_cell_dist(int32_t W, double s, int32_t a, int32_t b)
{
    double dx = (double)(b % W - a % W) * s, dy = (double)(b / W - a / W) * s;
    return sqrt(dx * dx + dy * dy);
}

/* Labelled pairs of one start: start id sid picks C-free cell
 * free_list[pick(w0)] with w = Philox(sid, 0, 0, 6).  For each bin k the goal
 * is, among C-free cells b valid with the start for bin k, the one with the
 * smallest (key, b), key = word 0 of Philox(sid, b, 0, 5): a uniform draw over
 * the bin's cells.  goal[k] = -1 and hops[k] = -1 for a bin with no cell.
 * Returns the start cell. */
int32_t orc_label_start(int32_t W, int32_t H, double s, const uint8_t *cfree,
                        const int32_t *free_list, int64_t nfree, const uint32_t key[2],
                        uint32_t sid, double d_lo, double d_hi, int32_t nbins, double gmd,
                        int32_t *goal, int32_t *hops)
{
    uint32_t w[4];
    orc_words(key, sid, 0u, 0u, 6u, w);
    int32_t a = free_list[orc_pick(w[0], nfree)];
    int64_t n = (int64_t)W * H;
    int32_t *field = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    orc_bfs_field(W, H, cfree, a, orc_max_hops(s, d_lo, d_hi, nbins), field);
    uint32_t *best = (uint32_t *)malloc((size_t)nbins * sizeof(uint32_t));
    for (int32_t k = 0; k < nbins; ++k) {
        goal[k] = -1;
        hops[k] = -1;
        best[k] = 0;
    }
    for (int64_t b = 0; b < n; ++b) {
        int32_t k = orc_bin_of(s, field[b], d_lo, d_hi, nbins);
        if (k < 0 || orc_cell_dist(W, s, a, (int32_t)b) < gmd) continue;
        orc_words(key, sid, (uint32_t)b, 0u, 5u, w);
        /* cells are visited in increasing b, so a strict < keeps the smaller b on ties */
        if (goal[k] < 0 || w[0] < best[k]) {
            best[k] = w[0];
            goal[k] = (int32_t)b;
            hops[k] = field[b];
        }
    }
    free(best);
    free(field);
    return a;
}

/* The exact check of a proposed pair for bin k.  Returns 1 when valid;
 * *hops_out = h(a, b) within the search depth, else -1. */
int32_t orc_verify_pair(int32_t W, int32_t H, double s, const uint8_t *cfree, int32_t a,
                        int32_t b, int32_t k, double d_lo, double d_hi, int32_t nbins, double gmd,
                        int32_t *hops_out)
{
    int64_t n = (int64_t)W * H;
    *hops_out = -1;
    if (a < 0 || a >= n || b < 0 || b >= n || !cfree[a] || !cfree[b]) return 0;
    int32_t *field = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    orc_bfs_field(W, H, cfree, a, orc_max_hops(s, d_lo, d_hi, nbins), field);
    *hops_out = field[b];
    free(field);
    if (orc_cell_dist(W, s, a, b) < gmd) return 0;
    return orc_bin_of(s, *hops_out, d_lo, d_hi, nbins) == k;
}

/* Plain rejection sampler for env e in episode ep asking for bin k: attempt t
 * draws w = Philox(e, ep, t, 7), start = free_list[pick(w0)], goal =
 * free_list[pick(w1)]; the first valid attempt wins.  Returns its index, or -1
 * after max_tries attempts (then *a_out = *b_out = -1). */
int32_t orc_reject_sample(int32_t W, int32_t H, double s, const uint8_t *cfree,
                          const int32_t *free_list, int64_t nfree, const uint32_t key[2],
                          uint32_t e, uint32_t ep, int32_t k, int32_t max_tries, double d_lo,
                          double d_hi, int32_t nbins, double gmd, int32_t *a_out, int32_t *b_out,
                          int32_t *hops_out, float *heading_out)
{
    *a_out = *b_out = *hops_out = -1;
    *heading_out = 0.0f;
    for (int32_t t = 0; t < max_tries; ++t) {
        uint32_t w[4];
        orc_words(key, e, ep, (uint32_t)t, 7u, w);
        int32_t a = free_list[orc_pick(w[0], nfree)], b = free_list[orc_pick(w[1], nfree)];
        int32_t h;
        *heading_out = (float)((((double)w[2] + 0.5) / 4294967296.0) * (2.0 * M_PI) - M_PI);
        if (orc_verify_pair(W, H, s, cfree, a, b, k, d_lo, d_hi, nbins, gmd, &h)) {
            *a_out = a;
            *b_out = b;
            *hops_out = h;
            return t;
        }
    }
    return -1;
}

/* Nearest C-free cell to cell c: least |di| + |dj|, ties to the least index;
 * -1 when the map has none. */
int32_t orc_snap_cell(int32_t W, int32_t H, const uint8_t *cfree, int32_t c)
{
    int32_t ci = c % W, cj = c / W, best = -1;
    int64_t bestd = 0;
    for (int64_t q = 0; q < (int64_t)W * H; ++q) {
        if (!cfree[q]) continue;
        int64_t d = llabs((int64_t)(q % W) - ci) + llabs((int64_t)(q / W) - cj);
        if (best < 0 || d < bestd) {
            best = (int32_t)q;
            bestd = d;
        }
    }
    return best;
}

/* 32 x 32 max-pooled occupancy of a W x H map (W, H >= 32): block (p, q)
 * covers columns [p W / 32, (p + 1) W / 32) and rows [q H / 32, (q + 1) H / 32)
 * (integer division); out[q 32 + p] = 1 when any cell of the block is occupied. */
void orc_pool32(int32_t W, int32_t H, const uint8_t *occ, float *out)
{
    for (int32_t q = 0; q < 32; ++q)
        for (int32_t p = 0; p < 32; ++p) {
            int32_t i0 = p * W / 32, i1 = (p + 1) * W / 32;
            int32_t j0 = q * H / 32, j1 = (q + 1) * H / 32;
            float v = 0.0f;
            for (int32_t j = j0; j < j1; ++j)
                for (int32_t i = i0; i < i1; ++i)
                    if (occ[(int64_t)j * W + i]) v = 1.0f;
            out[q * 32 + p] = v;
        }
}

/* Cells of a proposal from the network's outputs y = (start x, start y,
 * heading, goal x, goal y), positions as fractions of the map's width and
 * height: column = floor(y0 W) clamped to [0, W - 1], likewise the others;
 * heading = clamp(y2, -1, 1) pi. */
void orc_decode_proposal(int32_t W, int32_t H, const float y[5], int32_t *a, int32_t *b,
                         float *heading)
{
    double v[4] = {(double)y[0] * (double)W, (double)y[1] * (double)H, (double)y[3] * (double)W,
                   (double)y[4] * (double)H};
    int32_t lim[4] = {W - 1, H - 1, W - 1, H - 1};
    int32_t c[4];
    for (int i = 0; i < 4; ++i) {
        double f = floor(v[i]);
        c[i] = f < 0.0 ? 0 : (f > (double)lim[i] ? lim[i] : (int32_t)f);
        if (v[i] != v[i]) c[i] = 0; /* NaN */
    }
    *a = c[1] * W + c[0];
    *b = c[3] * W + c[2];
    double t = (double)y[2];
    t = t != t ? 0.0 : (t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t));
    *heading = (float)(t * 3.14159265358979323846);
}
