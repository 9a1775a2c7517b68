/*
 * Plain CPU oracle for the batched bitmap navigation step (FlashNav, arXiv
 * 2606.15846).  TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Everything is scalar double precision, evaluated in the order written here
 * (build with -ffp-contract=off so no multiply-add is fused).  State values are
 * float32; each one is read, widened exactly to double, and every stored
 * quantity is rounded once back to float32 (round to nearest even).
 *
 * What is computed, per environment and step (the step data path, eq. 7):
 *   action -> velocity command (section 2.2.3, table 7 normalised range),
 *   forward-Euler planar integration (section 2.2.3),
 *   footprint collision against the occupancy grid, out-of-bounds counting as
 *     occupied (section 2.2.1),
 *   K-beam range scan (eq. 4-5): the first occupied or out-of-bounds cell along
 *     each ray, found by an exact grid traversal (Amanatides & Woo), range =
 *     distance at which the ray enters that cell, clamped to r_max,
 *   sector min-pooling (eq. 6),
 *   relative goal distance and bearing in the robot frame (eq. 1),
 *   reward (eq. 3), termination and truncation (section 2.2.3),
 *   observation [l_1..l_m, d, phi, v, w] (eq. 1, raw pooled ranges),
 *   sparse reset of finished envs to collision-free start/goal poses with the
 *     final observation kept apart (section 2.2.3).
 * Readings where the paper is silent are listed beside each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF (1.0 / 0.0)

typedef struct {
    int32_t num_envs, num_beams, num_sectors;
    float fov_rad, max_range_m, dt_s;
    int32_t horizon;
    float goal_radius_m, c_progress, r_success, r_collision;
    int32_t footprint; /* 0 disc, 1 rectangle */
    float radius_m, length_m, width_m;
    float v_min, v_max, w_min, w_max;
    float goal_min_dist_m;
    int32_t reset_max_tries;
    uint64_t seed;
    int32_t scan_mode;  /* 0 exact grid traversal, 1 fixed-step march */
    float march_step_m; /* the march's sample spacing h */
} orc_cfg;

typedef struct {
    int32_t num_maps;
    const int32_t *w, *h;
    const float *res;
    const int64_t *off;        /* start of map k in occ */
    const uint8_t *occ;        /* row-major [h][w], nonzero = occupied */
    const int64_t *free_off;   /* start of map k's free-cell list */
    const int32_t *free_cnt;
    const int32_t *free_cells; /* iy*w + ix */
    /* optional per-map robot/sensor profile (NULL: the config's values) */
    const int32_t *prof_beams, *prof_footprint;
    const float *prof_radius, *prof_length, *prof_width;
} orc_maps;

typedef struct {
    float *x, *y, *th, *v, *w, *gx, *gy, *dprev;
    int32_t *t;
    uint32_t *ep;
    const int32_t *map;
} orc_state;

typedef struct {
    float *obs, *reward;
    uint8_t *terminated, *truncated;
    float *final_obs;
    float *ranges;     /* [N][K] scan of the pre-reset pose */
    int32_t *hits;     /* [N][K] hit cell iy*W+ix, -1 no hit, -2 map boundary */
    uint8_t *grazing;  /* [N][K] */
    int32_t *visits;   /* [N][K] cells whose occupancy the traversal read */
    uint8_t *collision, *goal, *reset, *fallback;
} orc_out;

typedef struct {
    double range, perp, t_end;
    int32_t hit, visits, grazing, pad;
} orc_ray;

/* The configuration that applies to envs on map `map`: the global one with
 * the map's beam count and footprint when a per-map profile is given. */
void orc_cfg_for_map(const orc_cfg *cfg, const orc_maps *M, int map, orc_cfg *out)
{
    *out = *cfg;
    if (M->prof_beams) out->num_beams = M->prof_beams[map];
    if (M->prof_footprint) {
        out->footprint = M->prof_footprint[map];
        out->radius_m = M->prof_radius[map];
        out->length_m = M->prof_length[map];
        out->width_m = M->prof_width[map];
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a counter-based        */
/* generator.  Ten rounds; each round multiplies words 0 and 2 by the two     */
/* round constants, mixes the high halves with the key and the other words,   */
/* and the key advances by the two Weyl constants between rounds.            */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform in (0, 1) from one 32-bit word: (w + 1/2) / 2^32, exact in double. */
static double orc_unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static void orc_draw(const orc_cfg *cfg, uint32_t env, uint32_t ep, uint32_t attempt,
                     uint32_t stream, double u[4])
{
    uint32_t ctr[4] = {env, ep, attempt, stream};
    uint32_t key[2] = {(uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = orc_unit(w[i]);
}

/* Synthetic rollout actions (the paper measures throughput under random
 * actions; the generator is this project's reading).  Env e at rollout step
 * n draws counter (e, n mod 2^32, n div 2^32, 4) and takes a_i = 2 u_i - 1
 * from the first two words, rounded once to float32; envs [e0, e1) go to
 * out[2 (e - e0) + i]. */
void orc_rollout_actions(const orc_cfg *cfg, uint64_t n, int64_t e0, int64_t e1, float *out)
{
    for (int64_t e = e0; e < e1; ++e) {
        double u[4];
        orc_draw(cfg, (uint32_t)e, (uint32_t)(n & 0xffffffffu), (uint32_t)(n >> 32), 4u, u);
        out[2 * (e - e0)] = (float)(2.0 * u[0] - 1.0);
        out[2 * (e - e0) + 1] = (float)(2.0 * u[1] - 1.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Grid (section 2.2.1): cell (i, j) is the box [i s, (i+1) s] x [j s, (j+1) s]; */
/* anything outside [0, W) x [0, H) counts as occupied.                         */
int orc_occupied(const orc_maps *M, int map, int64_t i, int64_t j)
{
    int64_t W = M->w[map], H = M->h[map];
    if (i < 0 || j < 0 || i >= W || j >= H) return 1;
    return M->occ[M->off[map] + j * W + i] != 0;
}

/* Disc of radius r at (x, y) against the grid: a cell collides when it is
 * occupied and its closest point lies strictly closer than r (touching is not
 * a collision). */
int orc_disc_hits(const orc_maps *M, int map, double x, double y, double r)
{
    double s = (double)M->res[map];
    int64_t i0 = (int64_t)floor((x - r) / s), i1 = (int64_t)floor((x + r) / s);
    int64_t j0 = (int64_t)floor((y - r) / s), j1 = (int64_t)floor((y + r) / s);
    double r2 = r * r;
    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            if (!orc_occupied(M, map, i, j)) continue;
            double bx0 = (double)i * s, bx1 = (double)(i + 1) * s;
            double by0 = (double)j * s, by1 = (double)(j + 1) * s;
            double cx = x < bx0 ? bx0 : (x > bx1 ? bx1 : x);
            double cy = y < by0 ? by0 : (y > by1 ? by1 : y);
            double ex = x - cx, ey = y - cy;
            if (ex * ex + ey * ey < r2) return 1;
        }
    }
    return 0;
}

/* Rectangle L x B centred at (x, y), long side along heading th.  A cell
 * collides when it is occupied and the separating-axis test finds strictly
 * overlapping projections on all four axes (x, y, heading, its normal). */
int orc_rect_hits(const orc_maps *M, int map, double x, double y, double th, double L, double B)
{
    double s = (double)M->res[map];
    double c = cos(th), sn = sin(th);
    double ac = fabs(c), as = fabs(sn);
    double hl = 0.5 * L, hb = 0.5 * B;
    double ex = hl * ac + hb * as;
    double ey = hl * as + hb * ac;
    double hs = 0.5 * s;
    double pu = hl + hs * (ac + as);
    double pw = hb + hs * (as + ac);
    int64_t i0 = (int64_t)floor((x - ex) / s), i1 = (int64_t)floor((x + ex) / s);
    int64_t j0 = (int64_t)floor((y - ey) / s), j1 = (int64_t)floor((y + ey) / s);
    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            if (!orc_occupied(M, map, i, j)) continue;
            double bx0 = (double)i * s, bx1 = (double)(i + 1) * s;
            double by0 = (double)j * s, by1 = (double)(j + 1) * s;
            if (!(x - ex < bx1 && bx0 < x + ex)) continue;
            if (!(y - ey < by1 && by0 < y + ey)) continue;
            double qx = (bx0 + hs) - x, qy = (by0 + hs) - y;
            double cu = qx * c + qy * sn;
            double cw = qy * c - qx * sn;
            if (fabs(cu) < pu && fabs(cw) < pw) return 1;
        }
    }
    return 0;
}

/* Radius of the disc that contains the footprint. */
double orc_circumradius(const orc_cfg *cfg)
{
    if (cfg->footprint == 0) return (double)cfg->radius_m;
    double hl = 0.5 * (double)cfg->length_m, hb = 0.5 * (double)cfg->width_m;
    return sqrt(hl * hl + hb * hb);
}

int orc_footprint_hits(const orc_maps *M, int map, const orc_cfg *cfg, double x, double y, double th)
{
    if (cfg->footprint == 0) return orc_disc_hits(M, map, x, y, (double)cfg->radius_m);
    return orc_rect_hits(M, map, x, y, th, (double)cfg->length_m, (double)cfg->width_m);
}

/* Free-cell list used when rejection sampling runs out of attempts: cells in
 * row-major order whose float32 centre passes the circumscribed-disc test. */
int64_t orc_free_list(const orc_maps *M, int map, double rc, int32_t *out)
{
    int64_t W = M->w[map], H = M->h[map];
    double s = (double)M->res[map];
    int64_t n = 0;
    for (int64_t j = 0; j < H; ++j) {
        for (int64_t i = 0; i < W; ++i) {
            float cx = (float)(((double)i + 0.5) * s);
            float cy = (float)(((double)j + 0.5) * s);
            if (!orc_disc_hits(M, map, (double)cx, (double)cy, rc)) {
                if (out) out[n] = (int32_t)(j * W + i);
                ++n;
            }
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* One ray (eq. 4): from (ox, oy) along unit (dx, dy).  Walks the cells the ray
 * passes through in order of entry distance; each boundary crossing distance is
 * recomputed from the integer cell index (never accumulated).  When the next x
 * and y crossings tie, the x crossing is taken first.  Stops at the first
 * occupied or out-of-bounds cell (range = its entry distance) or when the next
 * crossing lies beyond r_max (range = r_max, hit = -1).  An origin in an
 * occupied / out-of-bounds cell gives range 0.
 * Grazing bookkeeping: perp is the smallest distance between the ray and the
 * grid corner at any crossing decision; a ray is reported as grazing when that
 * is below eps, when its final crossing lies within eps of r_max, or when the
 * origin lies within eps of a grid line. */
void orc_cast(const orc_maps *M, int map, double ox, double oy, double dx, double dy,
              double rmax, double eps, orc_ray *r)
{
    int64_t W = M->w[map], H = M->h[map];
    double s = (double)M->res[map];
    int64_t i = (int64_t)floor(ox / s), j = (int64_t)floor(oy / s);
    double near = fmin(fmin(ox - (double)i * s, (double)(i + 1) * s - ox),
                       fmin(oy - (double)j * s, (double)(j + 1) * s - oy));
    r->perp = ORC_INF;
    r->visits = 1;
    r->t_end = 0.0;
    if (i < 0 || j < 0 || i >= W || j >= H) {
        r->range = 0.0;
        r->hit = -2;
        r->grazing = near < eps;
        return;
    }
    if (M->occ[M->off[map] + j * W + i]) {
        r->range = 0.0;
        r->hit = (int32_t)(j * W + i);
        r->grazing = near < eps;
        return;
    }
    int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1;
    double t;
    for (;;) {
        double tx = dx != 0.0 ? ((double)(i + (dx > 0.0 ? 1 : 0)) * s - ox) / dx : ORC_INF;
        double ty = dy != 0.0 ? ((double)(j + (dy > 0.0 ? 1 : 0)) * s - oy) / dy : ORC_INF;
        if (tx != ORC_INF && ty != ORC_INF) {
            double p = fabs(tx - ty) * fabs(dx * dy);
            if (p < r->perp) r->perp = p;
        }
        if (tx <= ty) {
            t = tx;
            i += sx;
        } else {
            t = ty;
            j += sy;
        }
        if (t > rmax) {
            r->range = rmax;
            r->hit = -1;
            break;
        }
        r->visits += 1;
        if (i < 0 || j < 0 || i >= W || j >= H) {
            r->range = t;
            r->hit = -2;
            break;
        }
        if (M->occ[M->off[map] + j * W + i]) {
            r->range = t;
            r->hit = (int32_t)(j * W + i);
            break;
        }
    }
    r->t_end = t;
    if (r->range < 0.0) r->range = 0.0;
    r->grazing = (r->perp < eps) || (fabs(t - rmax) < eps) || (near < eps);
}

/* The paper's own range query (section 2.2.2, table 7): sample the ray at a
 * fixed spacing h, tau_j = j h for j = 0, 1, ..., until the sample's cell is
 * occupied or out of bounds (range = tau_j) or tau_j exceeds r_max (range =
 * r_max).  Sampling can step over the corner of a cell the ray only clips.
 * Optional: *samples = samples evaluated, *near = least distance (in cells)
 * of an evaluated sample's coordinate to a grid line. */
void orc_march(const orc_maps *M, int map, double ox, double oy, double dx, double dy,
               double rmax, double h, double *range, int32_t *hit, int32_t *samples,
               double *near)
{
    int64_t W = M->w[map], H = M->h[map];
    double s = (double)M->res[map];
    double nr = 1.0;
    for (int64_t k = 0;; ++k) {
        double tau = (double)k * h;
        if (tau > rmax) {
            *range = rmax;
            *hit = -1;
            if (samples) *samples = (int32_t)k;
            break;
        }
        double px = ox + tau * dx, py = oy + tau * dy;
        double fx = px / s, fy = py / s;
        double gx = fabs(fx - nearbyint(fx)), gy = fabs(fy - nearbyint(fy));
        nr = gx < nr ? gx : nr;
        nr = gy < nr ? gy : nr;
        int64_t i = (int64_t)floor(fx), j = (int64_t)floor(fy);
        if (i < 0 || j < 0 || i >= W || j >= H) {
            *range = tau;
            *hit = -2;
            if (samples) *samples = (int32_t)(k + 1);
            break;
        }
        if (M->occ[M->off[map] + j * W + i]) {
            *range = tau;
            *hit = (int32_t)(j * W + i);
            if (samples) *samples = (int32_t)(k + 1);
            break;
        }
    }
    if (near) *near = nr;
}

/* Beam k's angle relative to the heading.  The paper only says the beams are
 * evenly spaced (appendix B); a full circle is split into K equal half-open
 * steps starting at -pi, a smaller field of view into K points including both
 * ends. */
double orc_beam_angle(const orc_cfg *cfg, int k)
{
    double fov = (double)cfg->fov_rad;
    int K = cfg->num_beams;
    if (fov >= 2.0 * M_PI - 1e-6) return -M_PI + (double)k * (2.0 * M_PI / (double)K);
    if (K == 1) return 0.0;
    return -0.5 * fov + (double)k * (fov / (double)(K - 1));
}

/* All K beams from pose (x, y, th). */
void orc_scan(const orc_maps *M, int map, const orc_cfg *cfg, double x, double y, double th,
              float *ranges, int32_t *hits, uint8_t *grazing, int32_t *visits)
{
    double rmax = (double)cfg->max_range_m;
    for (int k = 0; k < cfg->num_beams; ++k) {
        double psi = th + orc_beam_angle(cfg, k);
        if (cfg->scan_mode == 1) {
            /* grazing: a sample within 1e-9 cells of a grid line */
            double rg, nr;
            int32_t hit, ns;
            orc_march(M, map, x, y, cos(psi), sin(psi), rmax, (double)cfg->march_step_m, &rg,
                      &hit, &ns, &nr);
            if (ranges) ranges[k] = (float)rg;
            if (hits) hits[k] = hit;
            if (grazing) grazing[k] = (uint8_t)(nr < 1e-9);
            if (visits) visits[k] = ns;
            continue;
        }
        orc_ray r;
        orc_cast(M, map, x, y, cos(psi), sin(psi), rmax, 1e-6, &r);
        if (ranges) ranges[k] = (float)r.range;
        if (hits) hits[k] = r.hit;
        if (grazing) grazing[k] = (uint8_t)r.grazing;
        if (visits) visits[k] = r.visits;
    }
}

/* Observation from a pose: pooled ranges (eq. 6, contiguous sectors of K/m
 * beams), then goal distance and bearing in the robot frame (eq. 1), then the
 * velocity command.  Returns the float32 goal distance; *d64 gets the
 * unrounded one. */
static float orc_observe(const orc_maps *M, int map, const orc_cfg *cfg, double x, double y,
                         double th, double gx, double gy, float v, float w, float *obs,
                         float *ranges, int32_t *hits, uint8_t *grazing, int32_t *visits,
                         double *d64_out)
{
    int K = cfg->num_beams, m = cfg->num_sectors, per = K / m;
    float *rg = ranges;
    float local[4096];
    if (!rg) rg = local;
    orc_scan(M, map, cfg, x, y, th, rg, hits, grazing, visits);
    double ddx = gx - x, ddy = gy - y;
    double d64 = sqrt(ddx * ddx + ddy * ddy);
    double c = cos(th), sn = sin(th);
    double phi = atan2(-sn * ddx + c * ddy, c * ddx + sn * ddy);
    float d32 = (float)d64;
    if (obs) {
        for (int j = 0; j < m; ++j) {
            float l = rg[j * per];
            for (int q = 1; q < per; ++q)
                if (rg[j * per + q] < l) l = rg[j * per + q];
            obs[j] = l;
        }
        obs[m] = d32;
        obs[m + 1] = (float)phi;
        obs[m + 2] = v;
        obs[m + 3] = w;
    }
    if (d64_out) *d64_out = d64;
    return d32;
}

/* Sparse reset of env e (section 2.2.3): new collision-free start and goal
 * drawn from the map's free space, counters cleared, fresh observation.
 * Draws: attempt a of the start uses Philox counter (e, episode, a, 0) and
 * gives x = u0 W s, y = u1 H s, th = (2 u2 - 1) pi; the first pose whose
 * footprint is clear wins.  Goal attempt b uses counter (e, episode, b, 1);
 * the first goal whose circumscribed disc is clear and which lies at least
 * goal_min_dist from the start wins.  When every attempt fails, a cell of the
 * free-cell list is taken instead (index floor(u0 n_free), counter stream 2
 * for the start, 3 for the goal; the goal fallback ignores the distance). */
static void orc_reset_env(const orc_cfg *gcfg, const orc_maps *M, orc_state *st, int64_t e,
                          float *obs, uint8_t *fallback)
{
    int map = st->map[e];
    orc_cfg mcfg;
    orc_cfg_for_map(gcfg, M, map, &mcfg);
    const orc_cfg *cfg = &mcfg;
    uint32_t ep = st->ep[e];
    double s = (double)M->res[map];
    double Ws = (double)M->w[map] * s, Hs = (double)M->h[map] * s;
    int64_t W = M->w[map];
    int A = cfg->reset_max_tries;
    double rc = orc_circumradius(cfg);
    double gmd = (double)cfg->goal_min_dist_m;
    double u[4];
    float xs = 0, ys = 0, ths = 0, gx = 0, gy = 0;
    int ok = 0;
    uint8_t fb = 0;
    for (int a = 0; a < A && !ok; ++a) {
        orc_draw(cfg, (uint32_t)e, ep, (uint32_t)a, 0, u);
        xs = (float)(u[0] * Ws);
        ys = (float)(u[1] * Hs);
        ths = (float)((2.0 * u[2] - 1.0) * M_PI);
        ok = !orc_footprint_hits(M, map, cfg, (double)xs, (double)ys, (double)ths);
    }
    if (!ok) {
        orc_draw(cfg, (uint32_t)e, ep, 0, 2, u);
        int64_t n = M->free_cnt[map];
        int64_t idx = (int64_t)floor(u[0] * (double)n);
        int32_t cell = M->free_cells[M->free_off[map] + idx];
        xs = (float)(((double)(cell % W) + 0.5) * s);
        ys = (float)(((double)(cell / W) + 0.5) * s);
        ths = (float)((2.0 * u[2] - 1.0) * M_PI);
        fb |= 1;
    }
    ok = 0;
    for (int b = 0; b < A && !ok; ++b) {
        orc_draw(cfg, (uint32_t)e, ep, (uint32_t)b, 1, u);
        gx = (float)(u[0] * Ws);
        gy = (float)(u[1] * Hs);
        if (orc_disc_hits(M, map, (double)gx, (double)gy, rc)) continue;
        double ddx = (double)gx - (double)xs, ddy = (double)gy - (double)ys;
        ok = sqrt(ddx * ddx + ddy * ddy) >= gmd;
    }
    if (!ok) {
        orc_draw(cfg, (uint32_t)e, ep, 0, 3, u);
        int64_t n = M->free_cnt[map];
        int64_t idx = (int64_t)floor(u[0] * (double)n);
        int32_t cell = M->free_cells[M->free_off[map] + idx];
        gx = (float)(((double)(cell % W) + 0.5) * s);
        gy = (float)(((double)(cell / W) + 0.5) * s);
        fb |= 2;
    }
    st->x[e] = xs;
    st->y[e] = ys;
    st->th[e] = ths;
    st->v[e] = 0.0f;
    st->w[e] = 0.0f;
    st->gx[e] = gx;
    st->gy[e] = gy;
    st->t[e] = 0;
    st->ep[e] = ep + 1;
    int m = cfg->num_sectors;
    float d32 = orc_observe(M, map, cfg, (double)xs, (double)ys, (double)ths, (double)gx,
                            (double)gy, 0.0f, 0.0f, obs ? obs + e * (m + 4) : NULL, NULL, NULL,
                            NULL, NULL, NULL);
    st->dprev[e] = d32;
    if (fallback) fallback[e] = fb;
}

/* Reset every env whose mask byte is nonzero (mask NULL = all), envs [e0, e1). */
/* Reset of envs [e0, e1) with mask[e] != 0 (NULL = all) to given poses
 * pose[5 e ..] = (x, y, heading, goal x, goal y): the state and reset
 * observation of a reset (section 2.2.3) without the sampling. */
void orc_reset_to(const orc_cfg *gcfg, const orc_maps *M, orc_state *st, const uint8_t *mask,
                  const float *pose, float *obs, int64_t e0, int64_t e1)
{
    for (int64_t e = e0; e < e1; ++e) {
        if (mask && !mask[e]) continue;
        int map = st->map[e];
        orc_cfg mcfg;
        orc_cfg_for_map(gcfg, M, map, &mcfg);
        const float *q = pose + 5 * e;
        st->x[e] = q[0];
        st->y[e] = q[1];
        st->th[e] = q[2];
        st->v[e] = 0.0f;
        st->w[e] = 0.0f;
        st->gx[e] = q[3];
        st->gy[e] = q[4];
        st->t[e] = 0;
        st->ep[e] = st->ep[e] + 1;
        int m = mcfg.num_sectors;
        st->dprev[e] = orc_observe(M, map, &mcfg, (double)q[0], (double)q[1], (double)q[2],
                                   (double)q[3], (double)q[4], 0.0f, 0.0f,
                                   obs ? obs + e * (m + 4) : NULL, NULL, NULL, NULL, NULL, NULL);
    }
}

void orc_reset(const orc_cfg *cfg, const orc_maps *M, orc_state *st, const uint8_t *mask,
               float *obs, uint8_t *fallback, int64_t e0, int64_t e1)
{
    for (int64_t e = e0; e < e1; ++e) {
        if (mask && !mask[e]) continue;
        orc_reset_env(cfg, M, st, e, obs, fallback);
    }
}

/* One step of envs [e0, e1), in the order of the step data path (eq. 7).
 * defer_bin (may be NULL): an env that ends with defer_bin[e] >= 0 is not
 * reset here (its pair comes from the learned proposal, applied afterwards
 * with orc_reset_to or, where no valid pair was found, orc_reset). */
void orc_step_defer(const orc_cfg *gcfg, const orc_maps *M, orc_state *st, const float *act,
                    const orc_out *out, const int32_t *defer_bin, int64_t e0, int64_t e1)
{
    int K = gcfg->num_beams, m = gcfg->num_sectors; /* output strides: the largest K */
    double dt = (double)gcfg->dt_s;
    for (int64_t e = e0; e < e1; ++e) {
        int map = st->map[e];
        orc_cfg mcfg;
        orc_cfg_for_map(gcfg, M, map, &mcfg);
        const orc_cfg *cfg = &mcfg;
        /* action map (section 2.2.3, table 7): clip to [-1, 1], NaN -> 0 */
        double a0 = (double)act[2 * e], a1 = (double)act[2 * e + 1];
        if (a0 != a0) a0 = 0.0;
        if (a1 != a1) a1 = 0.0;
        a0 = a0 < -1.0 ? -1.0 : (a0 > 1.0 ? 1.0 : a0);
        a1 = a1 < -1.0 ? -1.0 : (a1 > 1.0 ? 1.0 : a1);
        double vlo = (double)cfg->v_min, vhi = (double)cfg->v_max;
        double wlo = (double)cfg->w_min, whi = (double)cfg->w_max;
        float v32 = (float)(vlo + ((a0 + 1.0) * 0.5) * (vhi - vlo));
        float w32 = (float)(wlo + ((a1 + 1.0) * 0.5) * (whi - wlo));
        /* forward Euler with the heading at the start of the step */
        double x = (double)st->x[e], y = (double)st->y[e], th = (double)st->th[e];
        double c = cos(th), sn = sin(th);
        double vdt = (double)v32 * dt;
        float x1 = (float)(x + vdt * c);
        float y1 = (float)(y + vdt * sn);
        double th2 = th + (double)w32 * dt;
        if (th2 >= M_PI)
            th2 -= 2.0 * M_PI;
        else if (th2 < -M_PI)
            th2 += 2.0 * M_PI;
        float th1 = (float)th2;
        /* collision at the new pose (the pose is kept even when it collides) */
        int coll = orc_footprint_hits(M, map, cfg, (double)x1, (double)y1, (double)th1);
        /* scan, pooling, goal features */
        float obs_row[4096 + 4];
        double d64;
        float d32 = orc_observe(M, map, cfg, (double)x1, (double)y1, (double)th1,
                                (double)st->gx[e], (double)st->gy[e], v32, w32, obs_row,
                                out->ranges ? out->ranges + e * K : NULL,
                                out->hits ? out->hits + e * K : NULL,
                                out->grazing ? out->grazing + e * K : NULL,
                                out->visits ? out->visits + e * K : NULL, &d64);
        /* reward (eq. 3) and episode flags */
        int goal = d64 < (double)cfg->goal_radius_m;
        int32_t t = st->t[e] + 1;
        int term = goal || coll;
        int trunc = (t >= cfg->horizon) && !term;
        float rew;
        if (goal)
            rew = cfg->r_success;
        else if (coll)
            rew = cfg->r_collision;
        else
            rew = (float)((double)cfg->c_progress * ((double)st->dprev[e] - (double)d32));
        st->x[e] = x1;
        st->y[e] = y1;
        st->th[e] = th1;
        st->v[e] = v32;
        st->w[e] = w32;
        st->dprev[e] = d32;
        st->t[e] = t;
        if (out->reward) out->reward[e] = rew;
        if (out->terminated) out->terminated[e] = (uint8_t)term;
        if (out->truncated) out->truncated[e] = (uint8_t)trunc;
        if (out->collision) out->collision[e] = (uint8_t)coll;
        if (out->goal) out->goal[e] = (uint8_t)goal;
        if (out->reset) out->reset[e] = (uint8_t)(term || trunc);
        if (out->fallback) out->fallback[e] = 0;
        if (out->obs) memcpy(out->obs + e * (m + 4), obs_row, sizeof(float) * (size_t)(m + 4));
        if (term || trunc) {
            if (out->final_obs)
                memcpy(out->final_obs + e * (m + 4), obs_row, sizeof(float) * (size_t)(m + 4));
            if (!(defer_bin && defer_bin[e] >= 0))
                orc_reset_env(gcfg, M, st, e, out->obs, out->fallback);
        }
    }
}

void orc_step(const orc_cfg *gcfg, const orc_maps *M, orc_state *st, const float *act,
              const orc_out *out, int64_t e0, int64_t e1)
{
    orc_step_defer(gcfg, M, st, act, out, NULL, e0, e1);
}
