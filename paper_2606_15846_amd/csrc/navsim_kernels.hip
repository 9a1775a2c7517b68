// HIP kernels of the batched bitmap navigation step (FlashNav, arXiv
// 2606.15846, section 2.2) for gfx950.
//
// Two mappings of the same step, with identical results:
//   fused_step_kernel  one workgroup per tile of envs sharing a map; the map's
//                      padded bitmap is staged once into LDS; one wavefront per
//                      env; lanes take beams (range scan), footprint cells
//                      (collision, ballot) and reset attempts (ballot, lowest
//                      successful attempt wins).
//   plain_step_kernel  one thread per env, everything sequential, bitmap read
//                      from device memory.  The comparison point.
//
// Numerics.  Per-env scalars (action map, kinematics, collision geometry, goal
// features, reward, reset draws) are evaluated in double precision in a fixed
// order with no fused multiply-add (the file is built with -ffp-contract=off);
// stored quantities are rounded once to float32.  Rays walk the grid with an
// exact integer decision variable: origin in 32.32 fixed point (cells),
// direction components |d| quantised to 2^-30.  The walk's cell order equals
// the exact ray's except for rays that pass within ~1e-8 cells of a grid corner.
#include <hip/hip_runtime.h>
#include <math.h>

#include "navsim_internal.hpp"

namespace navsim {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPow32 = 4294967296.0;
constexpr double kTwoPow30 = 1073741824.0;

// ---------------------------------------------------------------------------
// Counter-based generator for the reset draws: Philox4x32-10 (Salmon et al.,
// SC'11).  Counter (env, episode, attempt, stream), key = 64-bit seed.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Four uniforms in (0, 1): (w + 1/2) 2^-32, exact in double.
__device__ __forceinline__ void draw4(const StepParams &p, uint32_t env, uint32_t ep,
                                      uint32_t attempt, uint32_t stream, double u[4]) {
    uint32_t c[4] = {env, ep, attempt, stream};
    philox4x32_10(c, p.key0, p.key1);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ((double)c[i] + 0.5) * (1.0 / kTwoPow32);
}

// ---------------------------------------------------------------------------
// Occupancy access.  `bits` points at the map's padded bitmap (LDS in the fused
// step, device memory in the plain one); pitch = 32 * words per row.
struct MapView {
    const uint32_t *bits;
    int w, h, pitch;
    double s;
};

__device__ __forceinline__ bool cell_filled(const MapView &M, int i, int j) {
    if ((unsigned)i >= (unsigned)M.w || (unsigned)j >= (unsigned)M.h) return true;
    const int b = (j + 1) * M.pitch + (i + 1);
    return (M.bits[b >> 5] >> (b & 31)) & 1u;
}

// Disc of squared radius r2 at (x, y) against cell (i, j)'s closed box: the
// closest point of the box lies strictly inside the disc.
__device__ __forceinline__ bool disc_cell(double x, double y, double r2, int i, int j, double s) {
    const double bx0 = (double)i * s, bx1 = (double)(i + 1) * s;
    const double by0 = (double)j * s, by1 = (double)(j + 1) * s;
    const double cx = x < bx0 ? bx0 : (x > bx1 ? bx1 : x);
    const double cy = y < by0 ? by0 : (y > by1 ? by1 : y);
    const double ex = x - cx, ey = y - cy;
    return ex * ex + ey * ey < r2;
}

// Rectangle L x B centred at the pose, long side along the heading: separating
// axes x, y, heading u and its normal w; overlap must be strict on all four.
struct RectGeom {
    double c, sn, ex, ey, hs, pu, pw;
};

__device__ __forceinline__ RectGeom rect_geom(double th, double L, double B, double s) {
    RectGeom g;
    sincos(th, &g.sn, &g.c);
    const double ac = fabs(g.c), as = fabs(g.sn);
    const double hl = 0.5 * L, hb = 0.5 * B;
    g.ex = hl * ac + hb * as;
    g.ey = hl * as + hb * ac;
    g.hs = 0.5 * s;
    g.pu = hl + g.hs * (ac + as);
    g.pw = hb + g.hs * (as + ac);
    return g;
}

__device__ __forceinline__ bool rect_cell(const RectGeom &g, double x, double y, int i, int j,
                                          double s) {
    const double bx0 = (double)i * s, bx1 = (double)(i + 1) * s;
    const double by0 = (double)j * s, by1 = (double)(j + 1) * s;
    if (!(x - g.ex < bx1 && bx0 < x + g.ex)) return false;
    if (!(y - g.ey < by1 && by0 < y + g.ey)) return false;
    const double qx = (bx0 + g.hs) - x, qy = (by0 + g.hs) - y;
    const double cu = qx * g.c + qy * g.sn;
    const double cw = qy * g.c - qx * g.sn;
    return fabs(cu) < g.pu && fabs(cw) < g.pw;
}

// Candidate cells of a box of half-extents (ex, ey) around (x, y).
struct CellRange {
    int i0, j0, nx, ny;
};

__device__ __forceinline__ int clamp_cell(double v) {
    if (!(v == v)) return 0;
    v = fmin(fmax(v, -1048576.0), 1048576.0);
    return (int)v;
}

__device__ __forceinline__ CellRange cells_around(double x, double y, double ex, double ey,
                                                  double s) {
    CellRange r;
    r.i0 = clamp_cell(floor((x - ex) / s));
    r.j0 = clamp_cell(floor((y - ey) / s));
    const int i1 = clamp_cell(floor((x + ex) / s));
    const int j1 = clamp_cell(floor((y + ey) / s));
    r.nx = min(max(i1 - r.i0 + 1, 0), 64);
    r.ny = min(max(j1 - r.j0 + 1, 0), 64);
    return r;
}

// One lane tests a whole footprint (reset attempts, plain kernel).
__device__ bool disc_hits_serial(const MapView &M, double x, double y, double r) {
    const CellRange cr = cells_around(x, y, r, r, M.s);
    const double r2 = r * r;
    for (int dj = 0; dj < cr.ny; ++dj)
        for (int di = 0; di < cr.nx; ++di) {
            const int i = cr.i0 + di, j = cr.j0 + dj;
            if (cell_filled(M, i, j) && disc_cell(x, y, r2, i, j, M.s)) return true;
        }
    return false;
}

__device__ bool footprint_hits_serial(const MapView &M, const StepParams &p, double x, double y,
                                      double th) {
    if (p.footprint == NAVSIM_DISC) return disc_hits_serial(M, x, y, (double)p.radius);
    const RectGeom g = rect_geom(th, (double)p.len, (double)p.wid, M.s);
    const CellRange cr = cells_around(x, y, g.ex, g.ey, M.s);
    for (int dj = 0; dj < cr.ny; ++dj)
        for (int di = 0; di < cr.nx; ++di) {
            const int i = cr.i0 + di, j = cr.j0 + dj;
            if (cell_filled(M, i, j) && rect_cell(g, x, y, i, j, M.s)) return true;
        }
    return false;
}

// A wavefront tests one footprint: candidate cells spread over lanes, ballot.
__device__ bool footprint_hits_wave(const MapView &M, const StepParams &p, double x, double y,
                                    double th, int lane) {
    bool hit = false;
    if (p.footprint == NAVSIM_DISC) {
        const double r = (double)p.radius, r2 = r * r;
        const CellRange cr = cells_around(x, y, r, r, M.s);
        const int total = cr.nx * cr.ny;
        for (int c = lane; c < total; c += 64) {
            const int i = cr.i0 + c % cr.nx, j = cr.j0 + c / cr.nx;
            if (cell_filled(M, i, j) && disc_cell(x, y, r2, i, j, M.s)) hit = true;
        }
    } else {
        const RectGeom g = rect_geom(th, (double)p.len, (double)p.wid, M.s);
        const CellRange cr = cells_around(x, y, g.ex, g.ey, M.s);
        const int total = cr.nx * cr.ny;
        for (int c = lane; c < total; c += 64) {
            const int i = cr.i0 + c % cr.nx, j = cr.j0 + c / cr.nx;
            if (cell_filled(M, i, j) && rect_cell(g, x, y, i, j, M.s)) hit = true;
        }
    }
    return __ballot(hit) != 0ull;
}

// ---------------------------------------------------------------------------
// Range scan (eq. 4-5).  Per pose: the origin in cells, split into a 32.32
// fixed-point value; per ray: the walk over the cells the ray enters, in order,
// until an occupied (or padding = out-of-bounds) cell or the cell holding the
// r_max end point.
struct RayOrigin {
    double x, y, s, xc, yc;
    int64_t OX, OY;
    int i0, j0, blocked, block_hit;
};

__device__ __forceinline__ RayOrigin ray_origin(const MapView &M, double x, double y) {
    RayOrigin o;
    o.x = x;
    o.y = y;
    o.s = M.s;
    o.xc = x / M.s;
    o.yc = y / M.s;
    o.OX = 0;
    o.OY = 0;
    o.i0 = 0;
    o.j0 = 0;
    const double fi = floor(o.xc), fj = floor(o.yc);
    if (!(fi >= 0.0 && fi < (double)M.w && fj >= 0.0 && fj < (double)M.h)) {
        o.blocked = 1;
        o.block_hit = -2;
        return o;
    }
    o.i0 = (int)fi;
    o.j0 = (int)fj;
    if (cell_filled(M, o.i0, o.j0)) {
        o.blocked = 1;
        o.block_hit = o.j0 * M.w + o.i0;
        return o;
    }
    o.blocked = 0;
    o.block_hit = 0;
    o.OX = (int64_t)floor(o.xc * kTwoPow32);
    o.OY = (int64_t)floor(o.yc * kTwoPow32);
    return o;
}

// Walk one ray from a free origin cell.  With g = distance to the next grid
// line in the direction of travel (2^-32 cells) and D = quantised |direction|,
// E = gx DY - gy DX compares the two next crossing distances; an x crossing
// adds 2^32 DY, a y crossing subtracts 2^32 DX.  The low word of E never
// changes, so only the high word is carried; a tie (E == 0) crosses x first.
// The walk is bounded by the number of cells to the r_max end point; the hit
// range is recomputed once in double from the crossed grid line.
template <typename Bits>
__device__ __forceinline__ void cast_ray(Bits bits, int pitch, int W, int H, const RayOrigin &o,
                                         double dx, double dy, double rmax, double rmax_c,
                                         float &range, int &hit, int &visits) {
    const uint32_t DX = (uint32_t)rint(fabs(dx) * kTwoPow30);
    const uint32_t DY = (uint32_t)rint(fabs(dy) * kTwoPow30);
    const bool px = dx > 0.0, py = dy > 0.0;
    const uint32_t fx = (uint32_t)(uint64_t)o.OX, fy = (uint32_t)(uint64_t)o.OY;
    const uint64_t gx = px ? (4294967296ull - fx) : (uint64_t)fx;
    const uint64_t gy = py ? (4294967296ull - fy) : (uint64_t)fy;
    const int64_t E = (int64_t)(gx * (uint64_t)DY) - (int64_t)(gy * (uint64_t)DX);
    int Eh = (int)(E >> 32);
    const int thr = ((uint32_t)(uint64_t)E == 0u) ? 1 : 0;
    const double exc = fmin(fmax(o.xc + rmax_c * dx, -1048576.0), 1048576.0);
    const double eyc = fmin(fmax(o.yc + rmax_c * dy, -1048576.0), 1048576.0);
    const int n = abs((int)floor(exc) - o.i0) + abs((int)floor(eyc) - o.j0);
    int B = (o.j0 + 1) * pitch + (o.i0 + 1);
    const int incx = px ? 1 : -1, incy = py ? pitch : -pitch;
    const int dEx = (int)DY, dEy = -(int)DX;
    int k = 0;
    bool found = false, lastx = false;
    for (; k < n; ++k) {
        const bool xs = Eh < thr;
        B += xs ? incx : incy;
        Eh += xs ? dEx : dEy;
        if ((bits[B >> 5] >> (B & 31)) & 1u) {
            found = true;
            lastx = xs;
            break;
        }
    }
    if (found) {
        visits = k + 2;
        const int row = B / pitch, col = B - row * pitch;
        const int ix = col - 1, iy = row - 1;
        double t = lastx ? (((double)(px ? ix : ix + 1)) * o.s - o.x) / dx
                         : (((double)(py ? iy : iy + 1)) * o.s - o.y) / dy;
        t = fmin(fmax(t, 0.0), rmax);
        range = (float)t;
        hit = ((unsigned)ix < (unsigned)W && (unsigned)iy < (unsigned)H) ? iy * W + ix : -2;
    } else {
        visits = n + 1;
        range = (float)rmax;
        hit = -1;
    }
}

// ---------------------------------------------------------------------------
// Per-env scalar pieces (section 2.2.3; eq. 1, eq. 3).
struct Motion {
    float v, w, x1, y1, th1;
};

__device__ __forceinline__ Motion apply_action(const StepParams &p, float a0f, float a1f,
                                               float xf, float yf, float thf) {
    double a0 = (double)a0f, a1 = (double)a1f;
    if (a0 != a0) a0 = 0.0;
    if (a1 != a1) a1 = 0.0;
    a0 = a0 < -1.0 ? -1.0 : (a0 > 1.0 ? 1.0 : a0);
    a1 = a1 < -1.0 ? -1.0 : (a1 > 1.0 ? 1.0 : a1);
    const double vlo = (double)p.vlo, vhi = (double)p.vhi;
    const double wlo = (double)p.wlo, whi = (double)p.whi;
    Motion m;
    m.v = (float)(vlo + ((a0 + 1.0) * 0.5) * (vhi - vlo));
    m.w = (float)(wlo + ((a1 + 1.0) * 0.5) * (whi - wlo));
    const double x = (double)xf, y = (double)yf, th = (double)thf;
    double sn, c;
    sincos(th, &sn, &c);
    const double vdt = (double)m.v * (double)p.dt;
    m.x1 = (float)(x + vdt * c);
    m.y1 = (float)(y + vdt * sn);
    double th2 = th + (double)m.w * (double)p.dt;
    if (th2 >= kPi)
        th2 -= 2.0 * kPi;
    else if (th2 < -kPi)
        th2 += 2.0 * kPi;
    m.th1 = (float)th2;
    return m;
}

// Goal distance (unrounded and float32) and bearing in the robot frame.
__device__ __forceinline__ void goal_features(double x, double y, double c, double sn, float gx,
                                              float gy, double &d64, float &d32, float &phi32) {
    const double ddx = (double)gx - x, ddy = (double)gy - y;
    d64 = sqrt(ddx * ddx + ddy * ddy);
    const double phi = atan2(-sn * ddx + c * ddy, c * ddx + sn * ddy);
    d32 = (float)d64;
    phi32 = (float)phi;
}

__device__ __forceinline__ float uniform_pos(double u, double extent) {
    return (float)(u * extent);
}

__device__ __forceinline__ float uniform_heading(double u) {
    return (float)((2.0 * u - 1.0) * kPi);
}

__device__ __forceinline__ void free_cell_centre(const StepParams &p, const MapDesc &md, double u,
                                                 float &x, float &y) {
    const int64_t idx = (int64_t)floor(u * (double)md.free_cnt);
    const int32_t cell = p.free_cells[md.free_off + idx];
    const int ix = cell % md.w, iy = cell / md.w;
    x = (float)(((double)ix + 0.5) * (double)md.res);
    y = (float)(((double)iy + 0.5) * (double)md.res);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Fused mapping: one wavefront per env.

// Scan all K beams of a pose into s_rng (lane-strided beams).
__device__ void scan_wave(const StepParams &p, const MapView &M, const RayOrigin &o, double c,
                          double sn, int lane, float *s_rng, int64_t dbg_row) {
    const double rmax = (double)p.rmax, rmax_c = rmax / M.s;
    for (int kb = 0; kb < p.K; kb += 64) {
        const int k = kb + lane;
        if (k >= p.K) break;
        float rg;
        int hit, vis;
        if (o.blocked) {
            rg = 0.0f;
            hit = o.block_hit;
            vis = 1;
        } else {
            const double2 cs = p.beams[k];
            const double dx = c * cs.x - sn * cs.y;
            const double dy = sn * cs.x + c * cs.y;
            cast_ray(M.bits, M.pitch, M.w, M.h, o, dx, dy, rmax, rmax_c, rg, hit, vis);
        }
        s_rng[k] = rg;
        if (dbg_row >= 0) {
            if (p.d_ranges) p.d_ranges[dbg_row * p.K + k] = rg;
            if (p.d_hits) p.d_hits[dbg_row * p.K + k] = hit;
            if (p.d_visits) p.d_visits[dbg_row * p.K + k] = vis;
        }
    }
    wave_sync();
}

// Pooled sector j (eq. 6): min over its K/m contiguous beams.
__device__ __forceinline__ float pooled(const StepParams &p, const float *s_rng, int j) {
    const int per = p.K / p.m;
    float l = s_rng[j * per];
    for (int q = 1; q < per; ++q) l = fminf(l, s_rng[j * per + q]);
    return l;
}

// Sparse reset of env e (section 2.2.3): lane a tries attempt a; the lowest
// successful attempt wins, which is the first success of the sequential
// sampler.  Writes the new state and the reset observation row.
__device__ void reset_env_wave(const StepParams &p, const MapView &M, const MapDesc &md, int e,
                               int lane, float *s_rng, float *obs_row) {
    const uint32_t ep = p.st.ep[e];
    const double s = M.s, Ws = (double)md.w * s, Hs = (double)md.h * s;
    float xs = 0.0f, ys = 0.0f, ths = 0.0f, gx = 0.0f, gy = 0.0f;
    uint32_t fb = 0;
    bool found = false;
    for (int a0 = 0; a0 < p.tries && !found; a0 += 64) {
        const int a = a0 + lane;
        bool ok = false;
        float cx = 0.0f, cy = 0.0f, ct = 0.0f;
        if (a < p.tries) {
            double u[4];
            draw4(p, (uint32_t)e, ep, (uint32_t)a, 0u, u);
            cx = uniform_pos(u[0], Ws);
            cy = uniform_pos(u[1], Hs);
            ct = uniform_heading(u[2]);
            ok = !footprint_hits_serial(M, p, (double)cx, (double)cy, (double)ct);
        }
        const uint64_t b = __ballot(ok);
        if (b) {
            const int win = __ffsll((unsigned long long)b) - 1;
            xs = __shfl(cx, win);
            ys = __shfl(cy, win);
            ths = __shfl(ct, win);
            found = true;
        }
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 2u, u);
        free_cell_centre(p, md, u[0], xs, ys);
        ths = uniform_heading(u[2]);
        fb |= 1u;
    }
    found = false;
    const double gmd = (double)p.gmd;
    for (int b0 = 0; b0 < p.tries && !found; b0 += 64) {
        const int bq = b0 + lane;
        bool ok = false;
        float cx = 0.0f, cy = 0.0f;
        if (bq < p.tries) {
            double u[4];
            draw4(p, (uint32_t)e, ep, (uint32_t)bq, 1u, u);
            cx = uniform_pos(u[0], Ws);
            cy = uniform_pos(u[1], Hs);
            if (!disc_hits_serial(M, (double)cx, (double)cy, p.rc)) {
                const double ddx = (double)cx - (double)xs, ddy = (double)cy - (double)ys;
                ok = sqrt(ddx * ddx + ddy * ddy) >= gmd;
            }
        }
        const uint64_t b = __ballot(ok);
        if (b) {
            const int win = __ffsll((unsigned long long)b) - 1;
            gx = __shfl(cx, win);
            gy = __shfl(cy, win);
            found = true;
        }
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 3u, u);
        free_cell_centre(p, md, u[0], gx, gy);
        fb |= 2u;
    }
    // observation of the new pose
    double sn, c;
    sincos((double)ths, &sn, &c);
    const RayOrigin o = ray_origin(M, (double)xs, (double)ys);
    scan_wave(p, M, o, c, sn, lane, s_rng, -1);
    double d64;
    float d32, phi;
    goal_features((double)xs, (double)ys, c, sn, gx, gy, d64, d32, phi);
    for (int j = lane; j < p.m + 4; j += 64) {
        float val;
        if (j < p.m)
            val = pooled(p, s_rng, j);
        else if (j == p.m)
            val = d32;
        else if (j == p.m + 1)
            val = phi;
        else
            val = 0.0f;
        obs_row[j] = val;
    }
    if (lane == 0) {
        p.st.x[e] = xs;
        p.st.y[e] = ys;
        p.st.th[e] = ths;
        p.st.v[e] = 0.0f;
        p.st.w[e] = 0.0f;
        p.st.gx[e] = gx;
        p.st.gy[e] = gy;
        p.st.dprev[e] = d32;
        p.st.t[e] = 0;
        p.st.ep[e] = ep + 1u;
        if (p.d_fb) p.d_fb[e] = (uint8_t)fb;
    }
    wave_sync();
}

__device__ void env_step_wave(const StepParams &p, const MapView &M, const MapDesc &md, int e,
                              int lane, float *s_rng) {
    const int row = p.m + 4;
    float *obs_row = p.obs + (int64_t)e * row;
    if (p.mode == 1) {
        if (p.mask && !p.mask[e]) return;
        reset_env_wave(p, M, md, e, lane, s_rng, obs_row);
        return;
    }
    const Motion mo = apply_action(p, p.act[2 * (int64_t)e], p.act[2 * (int64_t)e + 1], p.st.x[e],
                                   p.st.y[e], p.st.th[e]);
    const double x1 = (double)mo.x1, y1 = (double)mo.y1, th1 = (double)mo.th1;
    const bool coll = footprint_hits_wave(M, p, x1, y1, th1, lane);
    double sn, c;
    sincos(th1, &sn, &c);
    const RayOrigin o = ray_origin(M, x1, y1);
    scan_wave(p, M, o, c, sn, lane, s_rng, e);
    double d64;
    float d32, phi;
    goal_features(x1, y1, c, sn, p.st.gx[e], p.st.gy[e], d64, d32, phi);
    const bool goal = d64 < (double)p.goal_r;
    const int t = p.st.t[e] + 1;
    const bool term = goal || coll;
    const bool trunc = (t >= p.horizon) && !term;
    const bool done = term || trunc;
    const float rew = goal ? p.r_succ
                           : (coll ? p.r_coll
                                   : (float)((double)p.c1 * ((double)p.st.dprev[e] - (double)d32)));
    float *fin = (done && p.final_obs) ? p.final_obs + (int64_t)e * row : nullptr;
    for (int j = lane; j < row; j += 64) {
        float val;
        if (j < p.m)
            val = pooled(p, s_rng, j);
        else if (j == p.m)
            val = d32;
        else if (j == p.m + 1)
            val = phi;
        else if (j == p.m + 2)
            val = mo.v;
        else
            val = mo.w;
        obs_row[j] = val;
        if (fin) fin[j] = val;
    }
    if (lane == 0) {
        p.reward[e] = rew;
        p.term[e] = (uint8_t)term;
        p.trunc[e] = (uint8_t)trunc;
        if (p.d_coll) p.d_coll[e] = (uint8_t)coll;
        if (p.d_goal) p.d_goal[e] = (uint8_t)goal;
        if (p.d_reset) p.d_reset[e] = (uint8_t)done;
        if (p.d_fb) p.d_fb[e] = 0;
        if (!done) {
            p.st.x[e] = mo.x1;
            p.st.y[e] = mo.y1;
            p.st.th[e] = mo.th1;
            p.st.v[e] = mo.v;
            p.st.w[e] = mo.w;
            p.st.dprev[e] = d32;
            p.st.t[e] = t;
        }
    }
    wave_sync();
    if (done) reset_env_wave(p, M, md, e, lane, s_rng, obs_row);
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void fused_step_kernel(StepParams p) {
    extern __shared__ uint4 smem4[];
    uint32_t *smem = reinterpret_cast<uint32_t *>(smem4);
    const Tile tile = p.tiles[blockIdx.x];
    const MapDesc md = p.maps[tile.map];
    const uint4 *src = reinterpret_cast<const uint4 *>(p.bits + md.word_off);
    for (int q = threadIdx.x; q < md.words / 4; q += WAVES * 64) smem4[q] = src[q];
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= tile.count) return;
    const int e = p.perm[tile.first + wave];
    float *s_rng = reinterpret_cast<float *>(smem + p.max_words) + wave * p.K;
    const MapView M{smem, md.w, md.h, md.wpr * 32, (double)md.res};
    env_step_wave(p, M, md, e, lane, s_rng);
}

// ---------------------------------------------------------------------------
// Plain mapping: one thread per env, the same arithmetic in sequence.

__device__ void observe_serial(const StepParams &p, const MapView &M, double x, double y, double c,
                               double sn, float *obs_row, int64_t dbg_row) {
    const RayOrigin o = ray_origin(M, x, y);
    const double rmax = (double)p.rmax, rmax_c = rmax / M.s;
    const int per = p.K / p.m;
    for (int j = 0; j < p.m; ++j) {
        float l = 0.0f;
        for (int q = 0; q < per; ++q) {
            const int k = j * per + q;
            float rg;
            int hit, vis;
            if (o.blocked) {
                rg = 0.0f;
                hit = o.block_hit;
                vis = 1;
            } else {
                const double2 cs = p.beams[k];
                const double dx = c * cs.x - sn * cs.y;
                const double dy = sn * cs.x + c * cs.y;
                cast_ray(M.bits, M.pitch, M.w, M.h, o, dx, dy, rmax, rmax_c, rg, hit, vis);
            }
            l = q == 0 ? rg : fminf(l, rg);
            if (dbg_row >= 0) {
                if (p.d_ranges) p.d_ranges[dbg_row * p.K + k] = rg;
                if (p.d_hits) p.d_hits[dbg_row * p.K + k] = hit;
                if (p.d_visits) p.d_visits[dbg_row * p.K + k] = vis;
            }
        }
        obs_row[j] = l;
    }
}

__device__ void reset_env_serial(const StepParams &p, const MapView &M, const MapDesc &md, int e,
                                 float *obs_row) {
    const uint32_t ep = p.st.ep[e];
    const double s = M.s, Ws = (double)md.w * s, Hs = (double)md.h * s;
    float xs = 0.0f, ys = 0.0f, ths = 0.0f, gx = 0.0f, gy = 0.0f;
    uint32_t fb = 0;
    bool found = false;
    for (int a = 0; a < p.tries && !found; ++a) {
        double u[4];
        draw4(p, (uint32_t)e, ep, (uint32_t)a, 0u, u);
        xs = uniform_pos(u[0], Ws);
        ys = uniform_pos(u[1], Hs);
        ths = uniform_heading(u[2]);
        found = !footprint_hits_serial(M, p, (double)xs, (double)ys, (double)ths);
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 2u, u);
        free_cell_centre(p, md, u[0], xs, ys);
        ths = uniform_heading(u[2]);
        fb |= 1u;
    }
    found = false;
    for (int b = 0; b < p.tries && !found; ++b) {
        double u[4];
        draw4(p, (uint32_t)e, ep, (uint32_t)b, 1u, u);
        gx = uniform_pos(u[0], Ws);
        gy = uniform_pos(u[1], Hs);
        if (disc_hits_serial(M, (double)gx, (double)gy, p.rc)) continue;
        const double ddx = (double)gx - (double)xs, ddy = (double)gy - (double)ys;
        found = sqrt(ddx * ddx + ddy * ddy) >= (double)p.gmd;
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 3u, u);
        free_cell_centre(p, md, u[0], gx, gy);
        fb |= 2u;
    }
    double sn, c;
    sincos((double)ths, &sn, &c);
    observe_serial(p, M, (double)xs, (double)ys, c, sn, obs_row, -1);
    double d64;
    float d32, phi;
    goal_features((double)xs, (double)ys, c, sn, gx, gy, d64, d32, phi);
    obs_row[p.m] = d32;
    obs_row[p.m + 1] = phi;
    obs_row[p.m + 2] = 0.0f;
    obs_row[p.m + 3] = 0.0f;
    p.st.x[e] = xs;
    p.st.y[e] = ys;
    p.st.th[e] = ths;
    p.st.v[e] = 0.0f;
    p.st.w[e] = 0.0f;
    p.st.gx[e] = gx;
    p.st.gy[e] = gy;
    p.st.dprev[e] = d32;
    p.st.t[e] = 0;
    p.st.ep[e] = ep + 1u;
    if (p.d_fb) p.d_fb[e] = (uint8_t)fb;
}

__global__ __launch_bounds__(64) void plain_step_kernel(StepParams p) {
    const int e = blockIdx.x * 64 + threadIdx.x;
    if (e >= p.N) return;
    const MapDesc md = p.maps[p.env_map[e]];
    const MapView M{p.bits + md.word_off, md.w, md.h, md.wpr * 32, (double)md.res};
    const int row = p.m + 4;
    float *obs_row = p.obs + (int64_t)e * row;
    if (p.mode == 1) {
        if (p.mask && !p.mask[e]) return;
        reset_env_serial(p, M, md, e, obs_row);
        return;
    }
    const Motion mo = apply_action(p, p.act[2 * (int64_t)e], p.act[2 * (int64_t)e + 1], p.st.x[e],
                                   p.st.y[e], p.st.th[e]);
    const double x1 = (double)mo.x1, y1 = (double)mo.y1, th1 = (double)mo.th1;
    const bool coll = footprint_hits_serial(M, p, x1, y1, th1);
    double sn, c;
    sincos(th1, &sn, &c);
    observe_serial(p, M, x1, y1, c, sn, obs_row, e);
    double d64;
    float d32, phi;
    goal_features(x1, y1, c, sn, p.st.gx[e], p.st.gy[e], d64, d32, phi);
    const bool goal = d64 < (double)p.goal_r;
    const int t = p.st.t[e] + 1;
    const bool term = goal || coll;
    const bool trunc = (t >= p.horizon) && !term;
    const bool done = term || trunc;
    const float rew = goal ? p.r_succ
                           : (coll ? p.r_coll
                                   : (float)((double)p.c1 * ((double)p.st.dprev[e] - (double)d32)));
    obs_row[p.m] = d32;
    obs_row[p.m + 1] = phi;
    obs_row[p.m + 2] = mo.v;
    obs_row[p.m + 3] = mo.w;
    if (done && p.final_obs) {
        float *fin = p.final_obs + (int64_t)e * row;
        for (int j = 0; j < row; ++j) fin[j] = obs_row[j];
    }
    p.reward[e] = rew;
    p.term[e] = (uint8_t)term;
    p.trunc[e] = (uint8_t)trunc;
    if (p.d_coll) p.d_coll[e] = (uint8_t)coll;
    if (p.d_goal) p.d_goal[e] = (uint8_t)goal;
    if (p.d_reset) p.d_reset[e] = (uint8_t)done;
    if (p.d_fb) p.d_fb[e] = 0;
    if (done) {
        reset_env_serial(p, M, md, e, obs_row);
    } else {
        p.st.x[e] = mo.x1;
        p.st.y[e] = mo.y1;
        p.st.th[e] = mo.th1;
        p.st.v[e] = mo.v;
        p.st.w[e] = mo.w;
        p.st.dprev[e] = d32;
        p.st.t[e] = t;
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_fused(const StepParams &p, hipStream_t s) {
    const size_t lds = (size_t)p.max_words * 4u + (size_t)kWavesPerGroup * (size_t)p.K * 4u;
    hipLaunchKernelGGL(fused_step_kernel<kWavesPerGroup>, dim3((unsigned)p.num_tiles),
                       dim3(kWavesPerGroup * 64), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_plain(const StepParams &p, hipStream_t s) {
    const unsigned blocks = (unsigned)((p.N + 63) / 64);
    hipLaunchKernelGGL(plain_step_kernel, dim3(blocks), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace navsim
