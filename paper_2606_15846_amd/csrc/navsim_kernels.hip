// HIP kernels of the batched bitmap navigation step (FlashNav, arXiv
// 2606.15846, section 2.2) for gfx950.
//
// Two mappings of the same step (step data path of eq. 7), identical results:
//   fused_step_kernel  one workgroup (256, 512 or 1024 threads) per tile of envs
//                      sharing a map: the map's padded bitmap (and, for the
//                      byte walks, a byte-per-cell copy) staged in LDS,
//                      per-env work on 16-lane groups, the tile's rays (new
//                      poses and reset poses) walked by all lanes from one
//                      refilling pool, set up and pooled either in bulk passes
//                      around the walk or by each lane as it claims and ends
//                      a ray, sector pooling in LDS.
//   plain_step_kernel  one thread per env, everything in sequence, bitmap read
//                      from device memory (the comparison point).
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

#include <algorithm>
#include <atomic>

#include "navsim_internal.hpp"
#include "philox.hpp"

namespace navsim {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPow32 = 4294967296.0;
constexpr double kTwoPow30 = 1073741824.0;

// Reset draws use Philox4x32-10 (philox.hpp) with counter (env, episode,
// attempt, stream) and key = 64-bit seed.
// Four uniforms in (0, 1): (w + 1/2) 2^-32, exact in double.
__device__ __forceinline__ void draw4(const StepParams &p, uint32_t env, uint32_t ep,
                                      uint32_t attempt, uint32_t stream, double u[4]) {
    uint32_t c[4] = {env, ep, attempt, stream};
    philox4x32_10(c, p.key0, p.key1);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ((double)c[i] + 0.5) * (1.0 / kTwoPow32);
}

// Normalised action of env e: the given one, or in a rollout the draw of
// counter (e, n mod 2^32, n div 2^32, 4) at step n, a_i = 2 u_i - 1.
__device__ __forceinline__ float2 env_action(const StepParams &p, int e) {
    if (!p.step_ctr) return make_float2(p.act[2 * (int64_t)e], p.act[2 * (int64_t)e + 1]);
    const uint64_t n = (((uint64_t)p.step_ctr[1] << 32) | (uint64_t)p.step_ctr[0]) +
                       (uint64_t)(uint32_t)p.step_off;
    double u[4];
    draw4(p, (uint32_t)e, (uint32_t)n, (uint32_t)(n >> 32), 4u, u);
    return make_float2((float)(2.0 * u[0] - 1.0), (float)(2.0 * u[1] - 1.0));
}

// ---------------------------------------------------------------------------
// Occupancy access.  `bits` points at the map's padded bitmap (LDS in the scan
// kernel, device memory elsewhere); pitch = 32 * wpr bits per padded row.
struct MapView {
    const uint32_t *bits;
    int w, h, wpr, pitch;
    double s;
    int pitch_t;                 // bits per line of the transposed bitmap
    float inv_pitch, inv_pitch_t;  // float reciprocals of the two (for small_divmod)
    uint32_t k_magic, per_magic;   // quotients by K and by beams per sector (MapDesc)
    int k_shift, per_shift;
};

__device__ __forceinline__ MapView map_view(const uint32_t *bits, const MapDesc &md) {
    const int pitch = md.wpr * 32, pitch_t = md.wpr_t * 32;
    return MapView{bits,         md.w,         md.h,
                   md.wpr,       pitch,        (double)md.res,
                   pitch_t,      __builtin_amdgcn_rcpf((float)pitch),
                   __builtin_amdgcn_rcpf((float)(pitch_t > 0 ? pitch_t : 1)),
                   md.k_magic,   md.per_magic, md.k_shift,
                   md.per_shift};
}

__device__ __forceinline__ bool cell_filled(const MapView &M, int i, int j) {
    if ((unsigned)i >= (unsigned)M.w || (unsigned)j >= (unsigned)M.h) return true;
    const int b = (j + kPad) * M.pitch + (i + kPad);
    return (M.bits[b >> 5] >> (b & 31)) & 1u;
}

// len (1..32) bits of padded row r starting at padded column c0, as the low
// bits of the result.
__device__ __forceinline__ uint32_t row_bits(const MapView &M, int r, int c0, int len) {
    const uint32_t *row = M.bits + r * M.wpr;
    const int w = c0 >> 5, sh = c0 & 31;
    uint64_t v = row[w];
    if (sh + len > 32) v |= (uint64_t)row[w + 1] << 32;
    const uint32_t bits = (uint32_t)(v >> sh);
    return len >= 32 ? bits : bits & ((1u << len) - 1u);
}

// Footprint of the robot on a map (per-map profile).
struct Robot {
    int footprint;
    double radius, len, wid, rc;
};

__device__ __forceinline__ Robot robot_of(const MapDesc &md) {
    return Robot{md.footprint, (double)md.radius, (double)md.len, (double)md.wid, md.rc};
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

__device__ __forceinline__ RectGeom rect_geom_cs(double c, double sn, double L, double B,
                                                 double s) {
    RectGeom g;
    g.c = c;
    g.sn = sn;
    const double ac = fabs(g.c), as = fabs(g.sn);
    const double hl = 0.5 * L, hb = 0.5 * B;
    g.ex = hl * ac + hb * as;
    g.ey = hl * as + hb * ac;
    g.hs = 0.5 * s;
    g.pu = hl + g.hs * (ac + as);
    g.pw = hb + g.hs * (as + ac);
    return g;
}

__device__ __forceinline__ RectGeom rect_geom(double th, double L, double B, double s) {
    double sn, c;
    sincos(th, &sn, &c);
    return rect_geom_cs(c, sn, L, B, s);
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
    // at most floor(2 ex / s) + 2 <= kMaxFootprintCells + 1 for a finite pose
    // (checked at load); the bound only stops runaway windows of garbage
    r.nx = min(max(i1 - r.i0 + 1, 0), 2 * kMaxFootprintCells);
    r.ny = min(max(j1 - r.j0 + 1, 0), 2 * kMaxFootprintCells);
    return r;
}

// Does any occupied candidate cell satisfy the exact predicate F(i, j)?  When
// the window lies inside the stored rows, whole rows are tested with one mask
// (four rows' masks read at a time, so their loads overlap) and F runs only on
// occupied cells; otherwise every cell is checked.  The answer does not depend
// on the order in which cells are tried.
template <typename F>
__device__ __forceinline__ bool any_filled_cell(const MapView &M, const CellRange &cr, F f) {
    const bool inside = cr.i0 >= -kPad && cr.j0 >= -kPad && cr.i0 + cr.nx <= M.w + kPad &&
                        cr.j0 + cr.ny <= M.h + kPad;
    if (inside) {
        const int r0 = cr.j0 + kPad, last = cr.ny - 1;
        for (int c = 0; c < cr.nx; c += 32) {
            const int c0 = cr.i0 + kPad + c, len = min(32, cr.nx - c);
            for (int dj = 0; dj < cr.ny; dj += 4) {
                uint32_t mk[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // rows past the window re-read its last row, then count as empty
                    const uint32_t v = row_bits(M, r0 + min(dj + q, last), c0, len);
                    mk[q] = dj + q <= last ? v : 0u;
                }
                if (!(mk[0] | mk[1] | mk[2] | mk[3])) continue;
                // one copy of the exact test for the four rows
#pragma unroll 1
                for (int q = 0; q < 4; ++q) {
                    uint32_t m = q == 0 ? mk[0] : (q == 1 ? mk[1] : (q == 2 ? mk[2] : mk[3]));
                    while (m) {
                        const int b = __ffs(m) - 1;
                        m &= m - 1u;
                        if (f(cr.i0 + c + b, cr.j0 + dj + q)) return true;
                    }
                }
            }
        }
        return false;
    }
    for (int dj = 0; dj < cr.ny; ++dj)
        for (int di = 0; di < cr.nx; ++di) {
            const int i = cr.i0 + di, j = cr.j0 + dj;
            if (cell_filled(M, i, j) && f(i, j)) return true;
        }
    return false;
}

__device__ bool disc_hits(const MapView &M, double x, double y, double r) {
    const CellRange cr = cells_around(x, y, r, r, M.s);
    const double r2 = r * r, s = M.s;
    return any_filled_cell(M, cr, [&](int i, int j) { return disc_cell(x, y, r2, i, j, s); });
}

__device__ bool footprint_hits_cs(const MapView &M, const Robot &rb, double x, double y,
                                  double c, double sn) {
    if (rb.footprint == NAVSIM_DISC) return disc_hits(M, x, y, rb.radius);
    const RectGeom g = rect_geom_cs(c, sn, rb.len, rb.wid, M.s);
    const CellRange cr = cells_around(x, y, g.ex, g.ey, M.s);
    const double s = M.s;
    return any_filled_cell(M, cr, [&](int i, int j) { return rect_cell(g, x, y, i, j, s); });
}

__device__ bool footprint_hits(const MapView &M, const Robot &rb, double x, double y, double th) {
    if (rb.footprint == NAVSIM_DISC) return disc_hits(M, x, y, rb.radius);
    double sn, c;
    sincos(th, &sn, &c);
    return footprint_hits_cs(M, rb, x, y, c, sn);
}

// ---------------------------------------------------------------------------
// Range scan (eq. 4-5).  Per pose: the origin in cells and its 32.32
// fixed-point value; per ray: a walk over the cells the ray enters, in order,
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

// r_max in cells for walk_setup, capped at kMaxWalkCells: a walk meets the
// padding ring within W + H + 2 kPad <= 8191 cells, so any budget beyond
// that is cut to the same walk, and the cap keeps the end point's cell index
// within int range.
constexpr double kMaxWalkCells = 16384.0;
__device__ __forceinline__ double walk_cells(double rmax, double s) {
    return fmin(rmax / s, kMaxWalkCells);
}

// Integer walk state of one ray.  With g = distance to the next grid line in
// the direction of travel (2^-32 cells) and D = quantised |direction|,
// E = gx DY - gy DX compares the two next crossing distances; an x crossing
// adds 2^32 DY, a y crossing subtracts 2^32 DX.  The low word of E never
// changes, so only the high word Eh is carried; a tie (E == 0) crosses x
// first.  n bounds the walk: cells between the origin and the r_max end point.
struct Walk {
    int B, Eh, thr, incx, incy, dEx, dEy, n;
};

__device__ __forceinline__ Walk walk_setup(int pitch, const RayOrigin &o, double dx, double dy,
                                           double rmax_c) {
    const uint32_t DX = (uint32_t)rint(fabs(dx) * kTwoPow30);
    const uint32_t DY = (uint32_t)rint(fabs(dy) * kTwoPow30);
    const bool px = dx > 0.0, py = dy > 0.0;
    const uint32_t fx = (uint32_t)(uint64_t)o.OX, fy = (uint32_t)(uint64_t)o.OY;
    // g = 2^32 - f or f: 33 bits (2^32 when f = 0 going up), taken as its low
    // word times D plus D 2^32 for that one case
    const uint32_t gxl = px ? 0u - fx : fx, gyl = py ? 0u - fy : fy;
    const uint64_t Px = (uint64_t)gxl * DY + ((px && fx == 0u) ? (uint64_t)DY << 32 : 0ull);
    const uint64_t Py = (uint64_t)gyl * DX + ((py && fy == 0u) ? (uint64_t)DX << 32 : 0ull);
    const int64_t E = (int64_t)(Px - Py);
    Walk w;
    w.Eh = (int)(E >> 32);
    w.thr = ((uint32_t)(uint64_t)E == 0u) ? 1 : 0;
    // rmax_c is at most kMaxWalkCells (see walk_cells) and the origin lies in
    // the map, so the end point converts to int without clamping
    const double exc = o.xc + rmax_c * dx;
    const double eyc = o.yc + rmax_c * dy;
    w.n = abs((int)floor(exc) - o.i0) + abs((int)floor(eyc) - o.j0);
    w.B = (o.j0 + kPad) * pitch + (o.i0 + kPad);
    w.incx = px ? 1 : -1;
    w.incy = py ? pitch : -pitch;
    w.dEx = (int)DY;
    w.dEy = -(int)DX;
    return w;
}

// q = floor(a / b) and r = a - q b for 0 <= a < 2^24, 1 <= b < 2^23 and
// a / b < 2^20, given inv_b within a few float ulps of 1 / b: the float
// estimate is then within one of the quotient, which the remainder (one
// full-rate 24-bit product) fixes.
__device__ __forceinline__ int small_divmod(int a, int b, float inv_b, int &r) {
    int q = (int)((float)a * inv_b);
    r = a - __mul24(q, b);
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    return q;
}

__device__ __forceinline__ int small_div(int a, int b, float inv_b) {
    int r;
    return small_divmod(a, b, inv_b, r);
}

// Sector of a beam: floor(beam / per) by one 24-bit product and a shift (the
// map's constants make it exact for every beam < 2^12).
__device__ __forceinline__ int beam_sector(const MapView &M, int beam) {
    return (int)(__umul24((uint32_t)beam, M.per_magic) >> M.per_shift);
}

// Job list entry and beam of claimed ray g = base + (lane's rank < 64), with
// base the same on every lane: one exact multiply-shift quotient of the
// uniform base (scalar), then at most one wrap per lane when K >= 64; smaller
// beam counts take the per-lane quotient.
__device__ __forceinline__ int claim_decode(const MapView &M, int base, int g, int K, float inv_K,
                                            int &beam) {
    if (K < 64) return small_divmod(g, K, inv_K, beam);
    // the constants are uniform: scalar registers, so that the product and
    // j0 K are scalar arithmetic
    const uint32_t km = __builtin_amdgcn_readfirstlane(M.k_magic);
    const uint32_t ks = __builtin_amdgcn_readfirstlane((uint32_t)M.k_shift);
    const int Ku = __builtin_amdgcn_readfirstlane(K);
    const int j0 = (int)(((uint64_t)(uint32_t)base * km) >> ks);
    beam = g - j0 * Ku;
    const bool wrap = beam >= Ku;
    beam -= wrap ? Ku : 0;
    return j0 + (wrap ? 1 : 0);
}

// Range and hit id of a walk that stopped in cell B.  The ray enters a cell
// when it has crossed both the cell's x line and its y line facing it, so the
// range is the later of the two crossing distances (a line behind the origin,
// or parallel to the ray, gives -inf); recomputed once in double.
__device__ __forceinline__ void walk_result(const RayOrigin &o, int pitch, float inv_pitch, int W,
                                            int H, int B, double dx, double dy, double rmax,
                                            float &range, int &hit, bool transposed = false) {
    // B: bit index of the cell in the bitmap (line = padded row, lines of
    // `pitch` bits), or in the transposed one (line = padded column)
    int pos;
    const int line = small_divmod(B, pitch, inv_pitch, pos);
    const int row = transposed ? pos : line, col = transposed ? line : pos;
    const int ix = col - kPad, iy = row - kPad;
    // t_x = X / dx and t_y = Y / dy (a zero component gives -inf); the later
    // one is picked without dividing, t_x > t_y iff X sgn(dx) |dy| > Y sgn(dy)
    // |dx| (both sides scaled by |dx| |dy| > 0), and only it is divided.  The
    // products can misorder the two only when they agree to ~1 ulp, i.e. for a
    // ray through a grid corner, and the value is then the same either way
    const double X = ((double)(dx > 0.0 ? ix : ix + 1)) * o.s - o.x;
    const double Y = ((double)(dy > 0.0 ? iy : iy + 1)) * o.s - o.y;
    const bool later_x = (dx > 0.0 ? X : -X) * fabs(dy) > (dy > 0.0 ? Y : -Y) * fabs(dx);
    const bool use_x = (dy == 0.0) | ((dx != 0.0) & later_x);
    // select first, then divide: one division per lane even when the lanes
    // of a wavefront pick different axes.  The quotient in single precision
    // (relative error about 2^-22: ~2 um at 8 m); its operands stay double,
    // since cancellation in X and Y is absolute, not relative
    const double num = use_x ? X : Y, den = use_x ? dx : dy;
    float t = (float)num * __builtin_amdgcn_rcpf((float)den);
    t = t > 0.0f ? t : 0.0f;  // also maps -0 and NaN to +0
    const float rm = (float)rmax;
    range = t < rm ? t : rm;
    hit = ((unsigned)ix < (unsigned)W && (unsigned)iy < (unsigned)H) ? __mul24(iy, W) + ix : -2;
}

// Sequential walk of one ray (plain kernel).
__device__ __forceinline__ void cast_ray(const MapView &M, const RayOrigin &o, double dx,
                                         double dy, double rmax, double rmax_c, float &range,
                                         int &hit, int &visits) {
    Walk w = walk_setup(M.pitch, o, dx, dy, rmax_c);
    int k = 0;
    bool found = false;
    while (k < w.n) {
        const bool xs = w.Eh < w.thr;
        w.B += xs ? w.incx : w.incy;
        w.Eh += xs ? w.dEx : w.dEy;
        ++k;
        if ((M.bits[w.B >> 5] >> (w.B & 31)) & 1u) {
            found = true;
            break;
        }
    }
    visits = k + 1;
    if (found) {
        walk_result(o, M.pitch, M.inv_pitch, M.w, M.h, w.B, dx, dy, rmax, range, hit);
    } else {
        range = (float)rmax;
        hit = -1;
    }
}

// Fixed-step march (the paper's range query, section 2.2.2, table 7): sample
// k at tau = k h, k = 0 .. march_kmax; returns 0 when the sample's cell is
// free, 1 occupied (cell id in *cell), 2 outside the map.  Cells come from
// floor(p / s) in double precision.
__device__ __forceinline__ int march_sample(const MapView &M, double x, double y, double dx,
                                            double dy, double h, int k, int *cell) {
    const double tau = (double)k * h;
    const double px = x + tau * dx, py = y + tau * dy;
    const double fi = floor(px / M.s), fj = floor(py / M.s);
    if (fi < 0.0 || fj < 0.0 || fi >= (double)M.w || fj >= (double)M.h) return 2;
    const int i = (int)fi, j = (int)fj;
    *cell = j * M.w + i;
    const int b = (j + kPad) * M.pitch + (i + kPad);
    return (int)((M.bits[b >> 5] >> (b & 31)) & 1u);
}

// Range, hit id and samples of a march that ended at sample k with outcome
// `type` (0: no hit up to k = march_kmax).
__device__ __forceinline__ void march_result(const StepParams &p, const MapView &M, double x,
                                             double y, double dx, double dy, int k, int type,
                                             float &range, int &hit, int &samples) {
    if (type == 0) {
        range = p.rmax;
        hit = -1;
        samples = p.march_kmax + 1;
        return;
    }
    range = (float)((double)k * p.march_h);
    samples = k + 1;
    if (type == 2) {
        hit = -2;
    } else {
        int cell = -1;
        (void)march_sample(M, x, y, dx, dy, p.march_h, k, &cell);
        hit = cell;
    }
}

__device__ __forceinline__ void march_ray(const StepParams &p, const MapView &M, double x,
                                          double y, double dx, double dy, float &range, int &hit,
                                          int &samples) {
    int k = 0, type = 0, cell = -1;
    for (; k <= p.march_kmax; ++k) {
        type = march_sample(M, x, y, dx, dy, p.march_h, k, &cell);
        if (type) break;
    }
    if (!type) k = p.march_kmax;
    march_result(p, M, x, y, dx, dy, k, type, range, hit, samples);
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

// Reset draws of env e (section 2.2.3): attempt a of the start pose uses
// counter (e, episode, a, 0), x = u0 W s, y = u1 H s, th = (2 u2 - 1) pi; the
// first pose whose footprint is clear wins.  Goal attempt b uses (e, episode,
// b, 1); the first goal whose circumscribed disc is clear and which is at
// least goal_min_dist from the start wins.  When all attempts fail, a cell of
// the free-cell list is used (stream 2 start, 3 goal).
struct ResetPose {
    float x, y, th, gx, gy;
    uint32_t fb;
};

__device__ ResetPose sample_reset(const StepParams &p, const MapView &M, const MapDesc &md,
                                  int e, uint32_t ep) {
    const double s = M.s, Ws = (double)md.w * s, Hs = (double)md.h * s;
    const Robot rb = robot_of(md);
    ResetPose r{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0u};
    bool found = false;
    for (int a = 0; a < p.tries && !found; ++a) {
        double u[4];
        draw4(p, (uint32_t)e, ep, (uint32_t)a, 0u, u);
        r.x = (float)(u[0] * Ws);
        r.y = (float)(u[1] * Hs);
        r.th = uniform_heading(u[2]);
        found = !footprint_hits(M, rb, (double)r.x, (double)r.y, (double)r.th);
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 2u, u);
        free_cell_centre(p, md, u[0], r.x, r.y);
        r.th = uniform_heading(u[2]);
        r.fb |= 1u;
    }
    found = false;
    for (int b = 0; b < p.tries && !found; ++b) {
        double u[4];
        draw4(p, (uint32_t)e, ep, (uint32_t)b, 1u, u);
        r.gx = (float)(u[0] * Ws);
        r.gy = (float)(u[1] * Hs);
        if (disc_hits(M, (double)r.gx, (double)r.gy, rb.rc)) continue;
        const double ddx = (double)r.gx - (double)r.x, ddy = (double)r.gy - (double)r.y;
        found = sqrt(ddx * ddx + ddy * ddy) >= (double)p.gmd;
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 3u, u);
        free_cell_centre(p, md, u[0], r.gx, r.gy);
        r.fb |= 2u;
    }
    return r;
}

// A reset pose supplied by the caller (row e of p.pose).
__device__ __forceinline__ ResetPose given_pose(const StepParams &p, int e) {
    const float *q = p.pose + 5 * (int64_t)e;
    ResetPose r;
    r.x = q[0];
    r.y = q[1];
    r.th = q[2];
    r.gx = q[3];
    r.gy = q[4];
    r.fb = 0u;
    return r;
}

// Store a reset: new state and the reset observation's scalar part (d, phi,
// v = w = 0); c, sn receive the new heading's cosine and sine for its scan.
__device__ void store_reset_cs(const StepParams &p, int e, uint32_t ep, const ResetPose &r,
                               double c, double sn) {
    double d64;
    float d32, phi;
    goal_features((double)r.x, (double)r.y, c, sn, r.gx, r.gy, d64, d32, phi);
    float *row = p.obs + (int64_t)e * (p.m + 4);
    row[p.m] = d32;
    row[p.m + 1] = phi;
    row[p.m + 2] = 0.0f;
    row[p.m + 3] = 0.0f;
    p.st.x[e] = r.x;
    p.st.y[e] = r.y;
    p.st.th[e] = r.th;
    p.st.v[e] = 0.0f;
    p.st.w[e] = 0.0f;
    p.st.gx[e] = r.gx;
    p.st.gy[e] = r.gy;
    p.st.dprev[e] = d32;
    p.st.t[e] = 0;
    p.st.ep[e] = ep + 1u;
    if (p.d_fb) p.d_fb[e] = (uint8_t)r.fb;
}

__device__ void store_reset(const StepParams &p, int e, uint32_t ep, const ResetPose &r,
                            double &c, double &sn) {
    sincos((double)r.th, &sn, &c);
    store_reset_cs(p, e, ep, r, c, sn);
}

// ---------------------------------------------------------------------------
// Fused step: one workgroup per tile of up to E envs that share a map.
//
//   1. stage the map's padded bitmap in LDS;
//   2. motion: a group of 16 lanes per env (action, kinematics, collision with
//      the footprint's candidate rows spread over the group, goal features,
//      reward, flags; for envs that ended, start and goal attempts on the
//      group's lanes, 8 + 8 in the first pass, then 16 of one kind at a time);
//   3. scan: the tile's pool of rays -- K per new pose and K per reset pose --
//      is walked by all lanes; a lane that finishes takes the next ray from an
//      LDS counter, refilled whenever at most refill_at lanes are busy, so the
//      lanes stay busy whatever the ray lengths;
//   4. sector minima (eq. 6) folded with LDS atomics, written as observation
//      rows.

struct TileJob {
    double c, s, x, y, xc, yc;
    int64_t OX, OY;
    int i0, j0, blocked, block_hit, env, dst;  // dst 0 obs row, 1 final_obs row, 2 none
    int B0, P0;  // the origin cell's bit index in the bitmap and in its transpose
};

// Register budget of the fused step: 4 wavefronts per SIMD (16 per CU).
constexpr int kFusedWavesPerSimd = 4;
constexpr int kGroupLanes = 16;

// Sector-pool words of a tile ([2E][m]), rounded up to keep the LDS regions
// after it 16-byte aligned.
__host__ __device__ constexpr int pool_words(int E, int m) { return (2 * E * m + 3) & ~3; }

size_t fused_lds_bytes(int max_words, int m, int E, int K, int ray_cap, int cell_bytes) {
    // K = 0 when the beam table stays in device memory
    return (size_t)max_words * 4u + (size_t)cell_bytes + 2u * (size_t)E * sizeof(TileJob) +
           (size_t)pool_words(E, m) * 4u + (4u * (size_t)E + 8u) * 4u + 16u * (size_t)K +
           16u * (size_t)ray_cap;
}

__device__ __forceinline__ void make_tile_job(TileJob &j, const MapView &M, float x, float y,
                                              double c, double s, int env, int dst) {
    const RayOrigin o = ray_origin(M, (double)x, (double)y);
    j.c = c;
    j.s = s;
    j.x = o.x;
    j.y = o.y;
    j.xc = o.xc;
    j.yc = o.yc;
    j.OX = o.OX;
    j.OY = o.OY;
    j.i0 = o.i0;
    j.j0 = o.j0;
    j.blocked = o.blocked;
    j.block_hit = o.block_hit;
    j.env = env;
    j.dst = dst;
    j.B0 = (o.j0 + kPad) * M.pitch + (o.i0 + kPad);
    j.P0 = (o.i0 + kPad) * M.pitch_t + (o.j0 + kPad);
}

// s_jobs[job], its offset as a full-rate 24-bit product (a TileJob's size is
// not a power of two)
__device__ __forceinline__ const TileJob &job_ref(const TileJob *s_jobs, int job) {
    return *reinterpret_cast<const TileJob *>(reinterpret_cast<const char *>(s_jobs) +
                                              __mul24(job, (int)sizeof(TileJob)));
}

__device__ __forceinline__ RayOrigin tile_origin(const TileJob &j, double s) {
    RayOrigin o;
    o.x = j.x;
    o.y = j.y;
    o.s = s;
    o.xc = j.xc;
    o.yc = j.yc;
    o.OX = j.OX;
    o.OY = j.OY;
    o.i0 = j.i0;
    o.j0 = j.j0;
    o.blocked = j.blocked;
    o.block_hit = j.block_hit;
    return o;
}

// Claim walks start on the main jobs' rays while the tile's reset poses are
// still being drawn; a reset job (index E + group) is published through the
// flag s_misc[2 + job] once its pose and walk origin are in s_jobs.  Reset
// rays come last in claim order, so the wait below is almost never taken; it
// ends because every listed reset job is drawn by its own group (bounded
// loops) before that group's wavefront enters the walk.
__device__ __forceinline__ void wait_job_ready(const int *s_misc, int job, int E) {
    if (job < E) return;
    while (__hip_atomic_load(s_misc + 2 + job, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
        __builtin_amdgcn_s_sleep(1);
}

// The 16 ballot bits of this lane's group of 16.
__device__ __forceinline__ uint32_t group_ballot(bool pred) {
    const uint64_t b = __ballot(pred);
    return (uint32_t)(b >> (threadIdx.x & 48)) & 0xFFFFu;
}

// Footprint test by a group of 16: lane li takes candidate rows li, li+16, ...
template <typename F>
__device__ __forceinline__ bool group_any_filled(const MapView &M, const CellRange &cr, int li,
                                                 F f) {
    const bool inside = cr.i0 >= -kPad && cr.j0 >= -kPad && cr.i0 + cr.nx <= M.w + kPad &&
                        cr.j0 + cr.ny <= M.h + kPad;
    bool hit = false;
    for (int dj = li; dj < cr.ny && !hit; dj += kGroupLanes) {
        if (inside) {
            const int r = cr.j0 + dj + kPad;
            for (int c = 0; c < cr.nx && !hit; c += 32) {
                uint32_t m = row_bits(M, r, cr.i0 + kPad + c, min(32, cr.nx - c));
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1u;
                    if (f(cr.i0 + c + b, cr.j0 + dj)) {
                        hit = true;
                        break;
                    }
                }
            }
        } else {
            for (int di = 0; di < cr.nx; ++di) {
                const int i = cr.i0 + di, j = cr.j0 + dj;
                if (cell_filled(M, i, j) && f(i, j)) {
                    hit = true;
                    break;
                }
            }
        }
    }
    return group_ballot(hit) != 0u;
}

__device__ bool group_footprint_hits(const MapView &M, const Robot &rb, double x, double y,
                                     double c, double sn, int li) {
    if (rb.footprint == NAVSIM_DISC) {
        const double r = rb.radius, r2 = r * r, s = M.s;
        const CellRange cr = cells_around(x, y, r, r, s);
        return group_any_filled(M, cr, li, [&](int i, int j) { return disc_cell(x, y, r2, i, j, s); });
    }
    const RectGeom g = rect_geom_cs(c, sn, rb.len, rb.wid, M.s);
    const CellRange cr = cells_around(x, y, g.ex, g.ey, M.s);
    const double s = M.s;
    return group_any_filled(M, cr, li, [&](int i, int j) { return rect_cell(g, x, y, i, j, s); });
}

// Reset draws of one env by its group of 16 lanes.  A goal's clearance test
// does not depend on the start pose (only its distance test does), so the
// first pass tests start attempts 0..7 on lanes 0..7 and goal attempts 0..7 on
// lanes 8..15 together; later passes test 16 attempts of one kind at a time.
// The lowest successful attempt of each kind wins, which is the first success
// of the sequential sampler.  c, sn receive the start heading's cosine and sine.
__device__ ResetPose group_sample_reset(const StepParams &p, const MapView &M, const MapDesc &md,
                                        int e, uint32_t ep, int li, double &c_out,
                                        double &sn_out) {
    constexpr int kHalf = kGroupLanes / 2;
    const double s = M.s, Ws = (double)md.w * s, Hs = (double)md.h * s;
    const Robot rb = robot_of(md);
    const int gbase = threadIdx.x & 48;
    ResetPose r{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0u};

    // ---- first pass: starts 0..7 and goals 0..7 ----
    const bool goal_lane = li >= kHalf;
    const int a1 = goal_lane ? li - kHalf : li;
    float fx = 0.0f, fy = 0.0f, ft = 0.0f;
    double fc = 1.0, fs = 0.0;
    bool clear = false;
    if (a1 < p.tries) {
        double u[4];
        draw4(p, (uint32_t)e, ep, (uint32_t)a1, goal_lane ? 1u : 0u, u);
        fx = (float)(u[0] * Ws);
        fy = (float)(u[1] * Hs);
        if (!goal_lane) {
            ft = uniform_heading(u[2]);
            sincos((double)ft, &fs, &fc);
        }
        bool hit;
        if (!goal_lane && rb.footprint != NAVSIM_DISC)
            hit = footprint_hits_cs(M, rb, (double)fx, (double)fy, fc, fs);
        else
            hit = disc_hits(M, (double)fx, (double)fy, goal_lane ? rb.rc : rb.radius);
        clear = !hit;
    }
    const uint32_t first = group_ballot(clear);
    bool found = false;
    if (first & 0xFFu) {
        const int src = gbase + __ffs(first & 0xFFu) - 1;
        r.x = __shfl(fx, src);
        r.y = __shfl(fy, src);
        r.th = __shfl(ft, src);
        c_out = __shfl(fc, src);
        sn_out = __shfl(fs, src);
        found = true;
    }
    for (int a0 = kHalf; a0 < p.tries && !found; a0 += kGroupLanes) {
        const int a = a0 + li;
        bool ok = false;
        float cx = 0.0f, cy = 0.0f, ct = 0.0f;
        double cc = 1.0, cs = 0.0;
        if (a < p.tries) {
            double u[4];
            draw4(p, (uint32_t)e, ep, (uint32_t)a, 0u, u);
            cx = (float)(u[0] * Ws);
            cy = (float)(u[1] * Hs);
            ct = uniform_heading(u[2]);
            sincos((double)ct, &cs, &cc);
            ok = !footprint_hits_cs(M, rb, (double)cx, (double)cy, cc, cs);
        }
        const uint32_t gm = group_ballot(ok);
        if (gm) {
            const int src = gbase + __ffs(gm) - 1;
            r.x = __shfl(cx, src);
            r.y = __shfl(cy, src);
            r.th = __shfl(ct, src);
            c_out = __shfl(cc, src);
            sn_out = __shfl(cs, src);
            found = true;
        }
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 2u, u);
        free_cell_centre(p, md, u[0], r.x, r.y);
        r.th = uniform_heading(u[2]);
        sincos((double)r.th, &sn_out, &c_out);
        r.fb |= 1u;
    }

    // ---- goals: the first pass's clear candidates, then 16 at a time ----
    const double gmd = (double)p.gmd;
    bool ok1 = false;
    if (goal_lane && clear) {
        const double ddx = (double)fx - (double)r.x, ddy = (double)fy - (double)r.y;
        ok1 = sqrt(ddx * ddx + ddy * ddy) >= gmd;
    }
    const uint32_t gm1 = group_ballot(ok1) >> kHalf;
    found = false;
    if (gm1) {
        const int src = gbase + kHalf + __ffs(gm1) - 1;
        r.gx = __shfl(fx, src);
        r.gy = __shfl(fy, src);
        found = true;
    }
    for (int b0 = kHalf; b0 < p.tries && !found; b0 += kGroupLanes) {
        const int b = b0 + li;
        bool ok = false;
        float cx = 0.0f, cy = 0.0f;
        if (b < p.tries) {
            double u[4];
            draw4(p, (uint32_t)e, ep, (uint32_t)b, 1u, u);
            cx = (float)(u[0] * Ws);
            cy = (float)(u[1] * Hs);
            if (!disc_hits(M, (double)cx, (double)cy, rb.rc)) {
                const double ddx = (double)cx - (double)r.x, ddy = (double)cy - (double)r.y;
                ok = sqrt(ddx * ddx + ddy * ddy) >= gmd;
            }
        }
        const uint32_t gm = group_ballot(ok);
        if (gm) {
            const int src = gbase + __ffs(gm) - 1;
            r.gx = __shfl(cx, src);
            r.gy = __shfl(cy, src);
            found = true;
        }
    }
    if (!found) {
        double u[4];
        draw4(p, (uint32_t)e, ep, 0u, 3u, u);
        free_cell_centre(p, md, u[0], r.gx, r.gy);
        r.fb |= 2u;
    }
    return r;
}

// Packed walk of one ray in LDS (16 bytes).  Written by the bulk setup:
//   x = B | n << 19        bit address of the origin cell, cells to walk
//   y = Eh - thr           the next crossing is an x crossing iff negative
//   z = DX | (dx > 0) << 31
//   w = DY | (dy > 0) << 31
// and, once walked, x = B | k << 19 (cell where the walk stopped, cells
// walked) and y = 1 if that cell is occupied.
__device__ __forceinline__ uint4 pack_walk(const Walk &w, int max_n) {
    const int n = min(w.n, max_n);
    uint4 r;
    r.x = (uint32_t)w.B | ((uint32_t)n << 19);
    r.y = (uint32_t)(w.Eh - w.thr);
    r.z = (uint32_t)(-w.dEy) | (w.incx > 0 ? 0x80000000u : 0u);
    r.w = (uint32_t)w.dEx | (w.incy > 0 ? 0x80000000u : 0u);
    return r;
}

// Range of a finished ray (direction dx, dy) folded into its sector's pooled
// minimum; per-ray outputs for main jobs when requested.
__device__ __forceinline__ void finish_ray_dir(const StepParams &p, const MapView &M,
                                               const TileJob &j, double dx, double dy, int job,
                                               int beam, uint2 res, uint32_t *s_pool, int per,
                                               float inv_per, int E) {
    float rg;
    int hit, vis;
    if (j.blocked) {
        rg = 0.0f;
        hit = j.block_hit;
        vis = 1;
    } else {
        const int B = (int)(res.x & 0x7FFFFu), k = (int)(res.x >> 19);
        vis = k + 1;
        if (res.y & 1u) {
            // bit 1: B indexes the transposed bitmap (run walk, y-major ray)
            const bool tr = (res.y & 2u) != 0u;
            walk_result(tile_origin(j, M.s), tr ? M.pitch_t : M.pitch,
                        tr ? M.inv_pitch_t : M.inv_pitch, M.w, M.h, B, dx, dy,
                        (double)p.rmax, rg, hit, tr);
        } else {
            rg = p.rmax;
            hit = -1;
        }
    }
    atomicMin(&s_pool[__mul24(job, p.m) + beam_sector(M, beam)], __float_as_uint(rg));
    if (job < E && (p.d_ranges || p.d_hits || p.d_visits)) {
        const int64_t o = (int64_t)j.env * p.K + beam;
        if (p.d_ranges) p.d_ranges[o] = rg;
        if (p.d_hits) p.d_hits[o] = hit;
        if (p.d_visits) p.d_visits[o] = vis;
    }
}

// The same with the direction recomputed from the job and the beam table.
__device__ __forceinline__ void finish_ray(const StepParams &p, const MapView &M, const TileJob &j,
                                           const double2 *s_beam, int job, int beam, uint2 res,
                                           uint32_t *s_pool, int per, float inv_per, int E) {
    double dx = 0.0, dy = 0.0;
    if (!j.blocked && (res.y & 1u)) {
        const double2 cs = s_beam[beam];
        dx = j.c * cs.x - j.s * cs.y;
        dy = j.s * cs.x + j.c * cs.y;
    }
    finish_ray_dir(p, M, j, dx, dy, job, beam, res, s_pool, per, inv_per, E);
}

// finish_ray for the fixed-step march: res.x = k | outcome << 28.
__device__ __forceinline__ void finish_march(const StepParams &p, const MapView &M,
                                             const TileJob &j, const double2 *s_beam, int job,
                                             int beam, uint32_t res, uint32_t *s_pool, int per,
                                             float inv_per, int E) {
    const double2 cs = s_beam[beam];
    const double dx = j.c * cs.x - j.s * cs.y;
    const double dy = j.s * cs.x + j.c * cs.y;
    float rg;
    int hit, vis;
    march_result(p, M, j.x, j.y, dx, dy, (int)(res & 0x0FFFFFFFu), (int)(res >> 28), rg, hit, vis);
    atomicMin(&s_pool[__mul24(job, p.m) + beam_sector(M, beam)], __float_as_uint(rg));
    if (job < E && (p.d_ranges || p.d_hits || p.d_visits)) {
        const int64_t o = (int64_t)j.env * p.K + beam;
        if (p.d_ranges) p.d_ranges[o] = rg;
        if (p.d_hits) p.d_hits[o] = hit;
        if (p.d_visits) p.d_visits[o] = vis;
    }
}

// Run walk (launch shape walk = 1): the same cell sequence as the 4-cell
// group walk, taken a run at a time.  Along the ray's major axis the cells
// between two minor-axis steps form a run; with E' the decision variable
// (x step iff E' < 0, +DY after an x step, -DX after a y step) a run's length
// follows from E' by one division for the first two runs and afterwards from
// the recurrence c = q + [v < r], v <- v - r + [v < r] Dmin (q, r: quotient
// and remainder of Dmaj / Dmin; v the residual of E' at the run's end), with
// no division.  A run along x is tested 32 cells at a time from a 64-bit
// window of two bitmap words (bit-reversed when walking toward -x), a run
// along y 4 cells at a time.
__device__ __forceinline__ int run_length(bool xmaj, int &Ep, int DX, int DY, int Dmin, int q,
                                          int rr, int &vv, int &exact, int rem) {
    if (exact > 0 || Dmin == 0) {
        int c;
        if (xmaj) {
            c = Ep < 0 ? (DY ? (int)(((uint32_t)(-Ep) + (uint32_t)DY - 1u) / (uint32_t)DY) : rem)
                       : 0;
            if (DY) Ep += c * DY;
        } else {
            c = Ep >= 0 ? (DX ? (int)((uint32_t)Ep / (uint32_t)DX) + 1 : rem) : 0;
            if (DX) Ep -= c * DX;
        }
        if (Dmin != 0 && --exact == 0) vv = xmaj ? Ep : -1 - Ep;
        return c;
    }
    const int b = vv < rr ? 1 : 0;
    vv = vv - rr + (b ? Dmin : 0);
    return q + b;
}

__device__ __forceinline__ void run_walk(const StepParams &p, const MapView &M,
                                         const uint32_t *s_bits, uint4 *s_ray, int *s_misc,
                                         int Rc, int lane) {
    int r = -1, B = 0, k = 0, rem = 0, Ep = 0, vv = 0, q = 0, rr = 0, Dmin = 0, DX = 0, DY = 0;
    int inc_maj = 0, inc_min = 0, exact = 0, cl = 0;
    bool act = false, exhausted = false, xmaj = false;
    uint32_t flags = 0u;
    for (;;) {
        uint64_t am = __ballot(act);
        if (!exhausted && __popcll(am) <= p.refill_at) {
            if (!act && r >= 0) {
                reinterpret_cast<uint2 *>(s_ray)[2 * r] =
                    make_uint2((uint32_t)B | ((uint32_t)k << 19), flags);
                r = -1;
            }
            const uint64_t idle = ~am;
            const int nidle = 64 - __popcll(am);
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_misc[1], nidle);
            // every lane is active here, so the first active one is lane 0
            base = __builtin_amdgcn_readfirstlane(base);
            const int my = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, (uint32_t)base));
            if (!act && my < Rc) {
                const uint4 v = s_ray[my];
                r = my;
                B = (int)(v.x & 0x7FFFFu);
                rem = (int)(v.x >> 19);
                Ep = (int)v.y;
                DX = (int)(v.z & 0x7FFFFFFFu);
                DY = (int)(v.w & 0x7FFFFFFFu);
                const int incx = (v.z >> 31) ? 1 : -1;
                const int incy = (v.w >> 31) ? M.pitch : -M.pitch;
                xmaj = DX >= DY;
                inc_maj = xmaj ? incx : incy;
                inc_min = xmaj ? incy : incx;
                Dmin = xmaj ? DY : DX;
                const int Dmaj = xmaj ? DX : DY;
                q = Dmin ? (int)((uint32_t)Dmaj / (uint32_t)Dmin) : 0;
                rr = Dmaj - q * Dmin;
                exact = 2;
                k = 0;
                flags = 0u;
                cl = run_length(xmaj, Ep, DX, DY, Dmin, q, rr, vv, exact, rem);
                act = rem > 0;
            }
            exhausted = base + nidle >= Rc;
            am = __ballot(act);
        }
        if (am == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (act) {
#pragma unroll 1
            for (int gi = 0; gi < p.groups; ++gi) {
                const int chunk = min(min(cl, rem), xmaj ? 32 : 4);
                uint32_t mk = 0u;
                if (chunk > 0) {
                    if (xmaj) {
                        if (inc_maj > 0) {
                            const int s0 = B + 1;
                            const uint64_t w = ((uint64_t)s_bits[(s0 >> 5) + 1] << 32) |
                                               (uint64_t)s_bits[s0 >> 5];
                            mk = (uint32_t)(w >> (s0 & 31));
                        } else {
                            const int e = B - 1;
                            const uint64_t w = ((uint64_t)s_bits[e >> 5] << 32) |
                                               (uint64_t)s_bits[(e >> 5) - 1];
                            mk = __brev((uint32_t)((w << (31 - (e & 31))) >> 32));
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int Bt = B + inc_maj * (t + 1);
                            mk |= ((s_bits[Bt >> 5] >> (Bt & 31)) & 1u) << t;
                        }
                    }
                    if (chunk < 32) mk &= (1u << chunk) - 1u;
                }
                if (mk) {
                    const int t = (int)__builtin_ctz(mk);
                    B += inc_maj * (t + 1);
                    k += t + 1;
                    flags = 1u;
                    act = false;
                    break;
                }
                B += inc_maj * chunk;
                k += chunk;
                rem -= chunk;
                cl -= chunk;
                if (rem <= 0) {
                    act = false;
                    break;
                }
                if (cl > 0) continue;
                // the minor-axis step that ends the run
                B += inc_min;
                k += 1;
                rem -= 1;
                if (exact > 0 || Dmin == 0) Ep = xmaj ? Ep - DX : Ep + DY;
                if ((s_bits[B >> 5] >> (B & 31)) & 1u) {
                    flags = 1u;
                    act = false;
                    break;
                }
                if (rem <= 0) {
                    act = false;
                    break;
                }
                cl = run_length(xmaj, Ep, DX, DY, Dmin, q, rr, vv, exact, rem);
            }
        }
    }
    if (r >= 0)
        reinterpret_cast<uint2 *>(s_ray)[2 * r] = make_uint2((uint32_t)B | ((uint32_t)k << 19), flags);
}

// Phase (2) for the fixed-step march: the refilling walk of the traversal
// with each lane marching its ray in groups of 4 samples (bitmap in LDS);
// the result k | outcome << 28 goes back to the ray's slot.
__device__ __forceinline__ void march_walk(const StepParams &p, const MapView &M,
                                           const TileJob *s_jobs, const int *s_list,
                                           const double2 *s_beam, uint4 *s_ray, int *s_misc,
                                           int c0, int Rc, int K, float inv_K, int lane) {
    int r = -1, k = 0, type = 0;
    bool act = false, exhausted = false;
    double x = 0.0, y = 0.0, dx = 0.0, dy = 0.0;
    const int kmax = p.march_kmax;
    const double h = p.march_h;
    for (;;) {
        uint64_t am = __ballot(act);
        if (!exhausted && __popcll(am) <= p.refill_at) {
            if (!act && r >= 0) {
                reinterpret_cast<uint2 *>(s_ray)[2 * r] =
                    make_uint2((uint32_t)k | ((uint32_t)type << 28), 0u);
                r = -1;
            }
            const uint64_t idle = ~am;
            const int nidle = 64 - __popcll(am);
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_misc[1], nidle);
            // every lane is active here, so the first active one is lane 0
            base = __builtin_amdgcn_readfirstlane(base);
            const int my = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, (uint32_t)base));
            if (!act && my < Rc) {
                const int g = c0 + my;
                int beam;
                const int jl = small_divmod(g, K, inv_K, beam);
                const TileJob &j = s_jobs[s_list[jl]];
                const double2 cs = s_beam[beam];
                dx = j.c * cs.x - j.s * cs.y;
                dy = j.s * cs.x + j.c * cs.y;
                x = j.x;
                y = j.y;
                r = my;
                k = 0;
                type = 0;
                act = true;
            }
            exhausted = base + nidle >= Rc;
            am = __ballot(act);
        }
        if (am == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (act) {
#pragma unroll 1
            for (int gi = 0; gi < p.groups; ++gi) {
                int cell, t[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    t[q] = (k + q <= kmax) ? march_sample(M, x, y, dx, dy, h, k + q, &cell) : 0;
                const int f = t[0] ? 0 : (t[1] ? 1 : (t[2] ? 2 : (t[3] ? 3 : 4)));
                if (f < 4) {
                    k += f;
                    type = t[f];
                    act = false;
                    break;
                }
                if (k + 3 >= kmax) {
                    k = kmax;
                    type = 0;
                    act = false;
                    break;
                }
                k += 4;
            }
        }
    }
    if (r >= 0)
        reinterpret_cast<uint2 *>(s_ray)[2 * r] = make_uint2((uint32_t)k | ((uint32_t)type << 28), 0u);
}

// Up to `groups` groups of 4 cells of one lane's walk; the 4 cells of a group
// are read before any is tested (the padding ring keeps them in the stored
// map).  Stops at the first occupied cell (flags = 1) or when the r_max
// budget n is used up; act turns false then.  The decision variable's high
// word and the cell index travel as one 64-bit value S = Eh : B, so a step is
// a compare, a 64-bit select and one 64-bit add: an x crossing adds
// Dx = dEx : incx and a y crossing Dy = dEy : incy (a negative increment
// borrows 1 from the high word, which the constant carries back; B + inc never
// leaves [0, 2^19), so each word gets exactly its own sum).
template <bool BYTES>
__device__ __forceinline__ void walk_groups(const StepParams &p, const uint32_t *s_bits,
                                            const uint8_t *s_cells, int &B, int &Eh, int incx,
                                            int incy, int dEx, int dEy, int n, int &k,
                                            uint32_t &flags, bool &act) {
    uint64_t S = ((uint64_t)(uint32_t)Eh << 32) | (uint64_t)(uint32_t)B;
    const uint64_t Dx = ((uint64_t)(uint32_t)dEx << 32) + (uint64_t)(int64_t)incx;
    const uint64_t Dy = ((uint64_t)(uint32_t)dEy << 32) + (uint64_t)(int64_t)incy;
#pragma unroll 1
    for (int gi = 0; gi < p.groups; ++gi) {
        const uint64_t S0 = S + ((int64_t)S < 0 ? Dx : Dy);
        const uint64_t S1 = S0 + ((int64_t)S0 < 0 ? Dx : Dy);
        const uint64_t S2 = S1 + ((int64_t)S1 < 0 ? Dx : Dy);
        const uint64_t S3 = S2 + ((int64_t)S2 < 0 ? Dx : Dy);
        const int B0 = (int)(uint32_t)S0, B1 = (int)(uint32_t)S1;
        const int B2 = (int)(uint32_t)S2, B3 = (int)(uint32_t)S3;
        uint32_t h;
        if (BYTES) {
            // one byte per cell at LDS address 0 (the kernel has no static
            // LDS, which the host checks): the cell index is the address
            typedef __attribute__((address_space(3))) const uint8_t lds_u8;
            const lds_u8 *cells = reinterpret_cast<const lds_u8 *>(static_cast<uintptr_t>(0));
            h = (uint32_t)cells[B0] | ((uint32_t)cells[B1] << 1) | ((uint32_t)cells[B2] << 2) |
                ((uint32_t)cells[B3] << 3);
        } else {
            const uint32_t w0 = s_bits[B0 >> 5], w1 = s_bits[B1 >> 5];
            const uint32_t w2 = s_bits[B2 >> 5], w3 = s_bits[B3 >> 5];
            h = __builtin_amdgcn_ubfe(w0, (uint32_t)B0, 1u) |
                (__builtin_amdgcn_ubfe(w1, (uint32_t)B1, 1u) << 1) |
                (__builtin_amdgcn_ubfe(w2, (uint32_t)B2, 1u) << 2) |
                (__builtin_amdgcn_ubfe(w3, (uint32_t)B3, 1u) << 3);
        }
        // first occupied cell of the group (4 when none); cells past
        // the r_max budget do not count
        const int rem = n - k;
        const int f = (int)__builtin_ctz(h | 16u);
        const bool hit = f < rem && f < 4;
        if (BYTES) {
            if (hit) {
                B = f == 0 ? B0 : (f == 1 ? B1 : (f == 2 ? B2 : B3));
                flags = 1u;
                k += f + 1;
                act = false;
                break;
            }
            if (rem <= 4) {
                k = n;
                act = false;
                break;
            }
        } else if (hit || rem <= 4) {
            // one exit (a hit, or the budget ends in this group): fewer
            // instructions per group in the bitmap walk (C4 641 -> 629 us); the
            // byte walk measured faster with the two exits above (C5 747 vs 754)
            if (hit) {
                B = f == 0 ? B0 : (f == 1 ? B1 : (f == 2 ? B2 : B3));
                flags = 1u;
                k += f + 1;
            } else {
                k = n;
            }
            act = false;
            break;
        }
        S = S3;
        B = B3;
        k += 4;
    }
    Eh = (int)(S >> 32);
}

// Up to `groups` groups of 4 cells of one lane's walk, for the claim walk:
// the state is S = Eh : B alone (an x crossing adds Dx = dEx : incx, a y
// crossing Dy = dEy : incy, see walk_groups) and the cells left in the r_max
// budget, rem.  One exit test per group: a cell of the group is occupied, or
// the budget ends in it; then the first occupied cell within the budget is
// the hit (Bh, flags = 1, rem reduced by the cells walked up to it), else
// the budget is used up (rem = 0); act turns false.
template <bool BYTES>
__device__ __forceinline__ void walk_run(const StepParams &p, const uint32_t *s_bits,
                                         uint64_t &S, uint64_t Dx, uint64_t Dy, int &rem,
                                         uint32_t &flags, bool &act, int &Bh) {
#pragma unroll 1
    for (int gi = 0; gi < p.groups; ++gi) {
        // the sign of S is the sign of its high word
        const uint64_t S0 = S + ((int)(uint32_t)(S >> 32) < 0 ? Dx : Dy);
        const uint64_t S1 = S0 + ((int)(uint32_t)(S0 >> 32) < 0 ? Dx : Dy);
        const uint64_t S2 = S1 + ((int)(uint32_t)(S1 >> 32) < 0 ? Dx : Dy);
        const uint64_t S3 = S2 + ((int)(uint32_t)(S2 >> 32) < 0 ? Dx : Dy);
        const int B0 = (int)(uint32_t)S0, B1 = (int)(uint32_t)S1;
        const int B2 = (int)(uint32_t)S2, B3 = (int)(uint32_t)S3;
        uint32_t h;
        if (BYTES) {
            typedef __attribute__((address_space(3))) const uint8_t lds_u8;
            const lds_u8 *cells = reinterpret_cast<const lds_u8 *>(static_cast<uintptr_t>(0));
            h = (uint32_t)cells[B0] | ((uint32_t)cells[B1] << 1) | ((uint32_t)cells[B2] << 2) |
                ((uint32_t)cells[B3] << 3);
        } else {
            const uint32_t w0 = s_bits[B0 >> 5], w1 = s_bits[B1 >> 5];
            const uint32_t w2 = s_bits[B2 >> 5], w3 = s_bits[B3 >> 5];
            h = __builtin_amdgcn_ubfe(w0, (uint32_t)B0, 1u) |
                (__builtin_amdgcn_ubfe(w1, (uint32_t)B1, 1u) << 1) |
                (__builtin_amdgcn_ubfe(w2, (uint32_t)B2, 1u) << 2) |
                (__builtin_amdgcn_ubfe(w3, (uint32_t)B3, 1u) << 3);
        }
        if (h != 0u || rem <= 4) {
            const int f = (int)__builtin_ctz(h | 16u);
            if (f < rem) {
                Bh = f == 0 ? B0 : (f == 1 ? B1 : (f == 2 ? B2 : B3));
                flags = 1u;
                rem -= f + 1;
            } else {
                rem = 0;
            }
            act = false;
            break;
        }
        S = S3;
        rem -= 4;
    }
}

// Group walk: lanes take rays from s_misc[1]; a lane whose ray is done
// writes its result back and takes a new one once at most refill_at lanes of
// its wavefront are still walking.  Cells are read from the bitmap, or (BYTES)
// from its one-byte-per-cell copy, which needs no address arithmetic or bit
// extraction; both give the same cells.
template <bool BYTES>
__device__ __forceinline__ void group_walk(const StepParams &p, const MapView &M,
                                           const uint32_t *s_bits, const uint8_t *s_cells,
                                           uint4 *s_ray, int *s_misc, int Rc, int lane) {
    int r = -1;
    bool act = false, exhausted = false;
    int B = 0, Eh = 0, incx = 0, incy = 0, dEx = 0, dEy = 0, n = 0, k = 0;
    uint32_t flags = 0u;
    for (;;) {
        uint64_t am = __ballot(act);
        if (!exhausted && __popcll(am) <= p.refill_at) {
            if (!act && r >= 0) {
                reinterpret_cast<uint2 *>(s_ray)[2 * r] =
                    make_uint2((uint32_t)B | ((uint32_t)k << 19), flags);
                r = -1;
            }
            const uint64_t idle = ~am;
            const int nidle = 64 - __popcll(am);
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_misc[1], nidle);
            // every lane is active here, so the first active one is lane 0
            base = __builtin_amdgcn_readfirstlane(base);
            const int my = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, (uint32_t)base));
            if (!act && my < Rc) {
                const uint4 v = s_ray[my];
                r = my;
                B = (int)(v.x & 0x7FFFFu);
                n = (int)(v.x >> 19);
                Eh = (int)v.y;
                dEy = -(int)(v.z & 0x7FFFFFFFu);
                dEx = (int)(v.w & 0x7FFFFFFFu);
                incx = (v.z >> 31) ? 1 : -1;
                incy = (v.w >> 31) ? M.pitch : -M.pitch;
                k = 0;
                flags = 0u;
                act = n > 0;
            }
            exhausted = base + nidle >= Rc;
            am = __ballot(act);
        }
        if (am == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (act)
            walk_groups<BYTES>(p, s_bits, s_cells, B, Eh, incx, incy, dEx, dEy, n, k, flags, act);
    }
    if (r >= 0)
        reinterpret_cast<uint2 *>(s_ray)[2 * r] = make_uint2((uint32_t)B | ((uint32_t)k << 19), flags);
}

// Claim walk: the group walk over all R rays of the tile, where a lane sets up
// the walk of each ray it claims (the job's origin, the rotated beam) and
// folds the ray's range into the sector pool once it is done.  The tile then
// needs no ray slots, no chunks and no separate setup and finish passes, and
// that work overlaps other wavefronts' walks.
template <bool BYTES>
__device__ __forceinline__ void claim_walk(const StepParams &p, const MapView &M,
                                           const uint32_t *s_bits, const uint8_t *s_cells,
                                           const TileJob *s_jobs, const int *s_list,
                                           const double2 *s_beam, uint32_t *s_pool, int *s_misc,
                                           int R, int K, float inv_K, int per, float inv_per,
                                           double rmax_c, int max_n, int E, int lane) {
    int g = -1, job = 0, beam = 0;
    bool act = false, exhausted = false;
    uint64_t S = 0, Dx = 0, Dy = 0;  // walk state and the two crossing steps (see walk_run)
    int n = 0, rem = 0, Bh = 0;
    uint32_t flags = 0u;
    double rdx = 0.0, rdy = 0.0;  // the claimed ray's direction, kept for its range
    for (;;) {
        uint64_t am = __ballot(act);
        if (!exhausted && __popcll(am) <= p.refill_at) {
            if (!act && g >= 0) {
                finish_ray_dir(p, M, job_ref(s_jobs, job), rdx, rdy, job, beam,
                               make_uint2((uint32_t)Bh | ((uint32_t)(n - rem) << 19), flags),
                               s_pool, per, inv_per, E);
                g = -1;
            }
            const uint64_t idle = ~am;
            const int nidle = 64 - __popcll(am);
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_misc[1], nidle);
            // every lane is active here, so the first active one is lane 0
            base = __builtin_amdgcn_readfirstlane(base);
            const int my = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, (uint32_t)base));
            if (!act && my < R) {
                g = my;
                const int jl = claim_decode(M, base, g, K, inv_K, beam);
                job = s_list[jl];
                wait_job_ready(s_misc, job, E);
                const TileJob &j = job_ref(s_jobs, job);
                n = 0;
                if (!j.blocked) {
                    const double2 cs = s_beam[beam];
                    rdx = j.c * cs.x - j.s * cs.y;
                    rdy = j.s * cs.x + j.c * cs.y;
                    const Walk w = walk_setup(M.pitch, tile_origin(j, M.s), rdx, rdy, rmax_c);
                    n = min(w.n, max_n);
                    S = ((uint64_t)(uint32_t)(w.Eh - w.thr) << 32) | (uint64_t)(uint32_t)w.B;
                    Dx = ((uint64_t)(uint32_t)w.dEx << 32) + (uint64_t)(int64_t)w.incx;
                    Dy = ((uint64_t)(uint32_t)w.dEy << 32) + (uint64_t)(int64_t)w.incy;
                }
                rem = n;
                flags = 0u;
                act = n > 0;
            }
            exhausted = base + nidle >= R;
            am = __ballot(act);
        }
        if (am == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (act) walk_run<BYTES>(p, s_bits, S, Dx, Dy, rem, flags, act, Bh);
    }
    if (g >= 0)
        finish_ray_dir(p, M, job_ref(s_jobs, job), rdx, rdy, job, beam,
                       make_uint2((uint32_t)Bh | ((uint32_t)(n - rem) << 19), flags), s_pool, per,
                       inv_per, E);
}

// Run walk on the bitmap and its transpose (walk 5).  Between two steps along
// its minor axis a ray moves along its major axis only, so its cells come in
// runs on one line of the map: a row of the bitmap for an x-major ray
// (DX >= DY), a row of the transposed bitmap (a column of the map) for a
// y-major one.  With e the decision variable of the integer walk turned so
// that a major step is taken iff e < 0 (x-major: e = E' as in walk_setup;
// y-major: e = -1 - E'), a major step adds a (the minor quantised component)
// and a minor step subtracts b (the major one).  Once e is in [0, a] (after
// the run that leaves the origin, which takes one division), every later run
// is a minor step and r = q + [e < M1] major steps with q = floor((b - 1) / a)
// and M1 = (b - 1) mod a + 1, after which e <- e - M1 + [e < M1] a stays in
// [0, a): runs of any length without dividing.  Up to 31 cells of a run are
// tested at once from two bitmap words (a funnel shift and a bit-field
// extract), so that lanes walking x- and y-major rays run the same
// instructions.  The cells, and therefore every result, are the other walks'.
constexpr int kLongRun = 1 << 14;  // run length of an axis-parallel ray (past any budget)

// floor(x / a) for 0 <= x <= 2^31 and 1 <= a <= 2^30 when that is below
// 12000, else kLongRun: a run that long outlasts any walk's budget (at most
// 8191 cells), so its exact length never matters.  a = 0 (inv_a infinite)
// also gives kLongRun.  inv_a is the float reciprocal of a; the float
// estimate is then within one of the quotient, and the two tests (q a < 2^32
// for such q) fix it.  r = x - q a when the quotient is returned (anything
// with kLongRun).  No branches: every lane of a refill takes the same path.
__device__ __forceinline__ int run_quot(uint32_t x, uint32_t a, float inv_a, uint32_t &r) {
    const float qf = (float)x * inv_a;
    const bool longr = !(qf < 12000.0f);
    const int q0 = (int)(longr ? 0.0f : qf);
    const uint32_t r0 = x - (uint32_t)q0 * a;
    const bool neg = (int32_t)r0 < 0;  // |r0| < 2 a <= 2^31: the sign bit tells
    const bool over = !neg && r0 >= a;
    r = neg ? r0 + a : (over ? r0 - a : r0);
    const int q = q0 + (over ? 1 : 0) - (neg ? 1 : 0);
    return longr ? kLongRun : q;
}

// Per-ray constants of the run walk.  Positions are bit indices into the
// staged line bitmap of the ray's major axis, plus `off`: the copy's start,
// and -31 when walking toward lower positions, so that a position is the
// first bit of the 32-cell window that holds the cell.
struct RunRay {
    int q1;         // q + 1: cells of a run without the extra major step
    int M1;         // e < M1 adds the extra major step
    int up, dn;     // e's change over a run: a - M1 with the extra step, -M1 without
    int dmin;       // a minor step relative to a major one
    int sm;         // 0 walking toward higher positions (a major step is +1), -1 toward lower
    int off;
};

// Up to `groups` windows of one lane's run walk.  State: X (the window
// position of the next cell along the major axis), e, pend (cells left in the
// current run, its minor step included) and rem (cells left in the r_max
// budget).  A window holds L = min(pend, rem, 31) cells; when one of them is
// occupied the first in walk order is the hit (Xh = its window position,
// flags = 1, rem reduced by the cells walked up to it), and when the budget
// ends in the window without a hit rem = 0; act turns false then.
__device__ __forceinline__ void run_windows(const StepParams &p, const uint32_t *s_bits,
                                            const RunRay &c, int &X, int &e, int &pend, int &rem,
                                            uint32_t &flags, bool &act, int &Xh) {
    uint32_t t = 0u;
    int Q = 0, L = 0;
    // one exit condition inside the loop (fewer lane masks to keep); the walk's
    // end is worked out after it from the last window
#pragma unroll 1
    for (int gi = 0; gi < p.groups; ++gi) {
        const bool newl = pend == 0;
        const bool extra = e < c.M1;
        pend = newl ? c.q1 + (int)extra : pend;
        e = newl ? e + (extra ? c.up : c.dn) : e;
        Q = X + (newl ? c.dmin : 0);
        L = min(min(pend, rem), 31);
        const int wq = Q >> 5;
        const uint32_t v = __builtin_amdgcn_alignbit(s_bits[wq + 1], s_bits[wq], (uint32_t)Q);
        // the window's cells: bits 0 .. L-1 walking up, 32-L .. 31 walking down
        t = __builtin_amdgcn_ubfe(v, (uint32_t)((32 - L) & c.sm), (uint32_t)L);
        // past the window (taken back below when the walk ends in it)
        X = Q + ((L ^ c.sm) - c.sm);
        pend -= L;
        rem -= L;
        if (t != 0u || rem <= 0) break;
    }
    if (t != 0u) {
        // walking up: the lowest set bit; walking down: the highest
        const int f = c.sm ? L - 32 + (int)__builtin_clz(t) : (int)__builtin_ctz(t);
        Xh = Q + ((f ^ c.sm) - c.sm);
        flags = 1u;
        rem += L - f - 1;
        act = false;
    } else if (rem <= 0) {
        rem = 0;
        act = false;
    }
}

// The claim walk (see claim_walk) over runs: each claimed ray is set up for
// run_windows, and a hit found in the transposed bitmap is turned back into
// the bitmap's cell index for walk_result.
__device__ __forceinline__ void claim_run_walk(const StepParams &p, const MapView &M,
                                               const uint32_t *s_bits,
                                               const TileJob *s_jobs, const int *s_list,
                                               const double2 *s_beam, uint32_t *s_pool,
                                               int *s_misc, int R, int K, float inv_K, int per,
                                               float inv_per, double rmax_c, int max_n, int E,
                                               int lane) {
    const int pitch_t = M.pitch_t;
    int g = -1, job = 0, beam = 0;
    bool act = false, exhausted = false, xmaj = true;
    RunRay c{};
    int X = 0, e = 0, pend = 0, n = 0, rem = 0, Xh = 0;
    uint32_t flags = 0u;
    double rdx = 0.0, rdy = 0.0;  // the claimed ray's direction, kept for its range
    auto finish = [&]() {
        // the hit's line position (0 without a hit: the field shares its word
        // with the visit count); flag bit 1 marks a position in the transpose
        const int Bh = flags ? Xh - c.off : 0;
        finish_ray_dir(p, M, job_ref(s_jobs, job), rdx, rdy, job, beam,
                       make_uint2((uint32_t)Bh | ((uint32_t)(n - rem) << 19),
                                  flags | (flags && !xmaj ? 2u : 0u)),
                       s_pool, per, inv_per, E);
    };
    for (;;) {
        uint64_t am = __ballot(act);
        if (!exhausted && __popcll(am) <= p.refill_at) {
            if (!act && g >= 0) {
                finish();
                g = -1;
            }
            const uint64_t idle = ~am;
            const int nidle = 64 - __popcll(am);
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_misc[1], nidle);
            // every lane is active here, so the first active one is lane 0
            base = __builtin_amdgcn_readfirstlane(base);
            const int my = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, (uint32_t)base));
            if (!act && my < R) {
                g = my;
                const int jl = claim_decode(M, base, g, K, inv_K, beam);
                job = s_list[jl];
                wait_job_ready(s_misc, job, E);
                const TileJob &j = job_ref(s_jobs, job);
                n = 0;
                if (!j.blocked) {
                    const double2 cs = s_beam[beam];
                    rdx = j.c * cs.x - j.s * cs.y;
                    rdy = j.s * cs.x + j.c * cs.y;
                    const Walk w = walk_setup(M.pitch, tile_origin(j, M.s), rdx, rdy, rmax_c);
                    n = min(w.n, max_n);
                    const int Ep = w.Eh - w.thr;  // x step iff Ep < 0
                    const int DX = -w.dEy, DY = w.dEx;
                    xmaj = DX >= DY;
                    const int a = xmaj ? DY : DX, b = xmaj ? DX : DY;
                    e = xmaj ? Ep : -1 - Ep;
                    // the run leaving the origin: ceil(-e / a) major steps; then
                    // q = floor((b - 1) / a) (a = 0: an axis-parallel ray, one run)
                    // (remainders instead of products: e + pend a = a - 1 - r0 and
                    // M1 = b - q a = r1 + 1)
                    // (a = 0, an axis-parallel ray: both quotients are kLongRun, one
                    // run, and e, M1 never matter; with e >= 0 the first step is the
                    // minor one and the first quotient is not used)
                    const float inv_a = __builtin_amdgcn_rcpf((float)a);
                    uint32_t r0 = 0u, r1 = 0u;
                    const int p0 = run_quot((uint32_t)(-e) + (uint32_t)(a - 1), (uint32_t)a, inv_a,
                                            r0);
                    const int q = run_quot((uint32_t)(b - 1), (uint32_t)a, inv_a, r1);
                    pend = e < 0 ? p0 : 0;
                    e = e < 0 ? a - 1 - (int)r0 : e;
                    c.q1 = q + 1;
                    c.M1 = (int)r1 + 1;
                    c.up = a - c.M1;
                    c.dn = -c.M1;
                    const bool down = xmaj ? w.incx < 0 : w.incy < 0;
                    const int smaj = down ? -1 : 1;
                    const int smin = xmaj ? w.incy : (w.incx > 0 ? pitch_t : -pitch_t);
                    c.sm = down ? -1 : 0;
                    c.dmin = smin - smaj;
                    c.off = (down ? -31 : 0) + (xmaj ? 0 : 32 * p.tbits_off);
                    X = (xmaj ? j.B0 : j.P0) + smaj + c.off;
                }
                rem = n;
                flags = 0u;
                act = n > 0;
            }
            exhausted = base + nidle >= R;
            am = __ballot(act);
        }
        if (am == 0ull) {
            if (exhausted) break;
            continue;
        }
        if (act) run_windows(p, s_bits, c, X, e, pend, rem, flags, act, Xh);
    }
    if (g >= 0) finish();
}

// LDS of the fused step, in order: the map's byte-per-cell copy [cell_bytes]
// (byte walk only: at address 0, so that a cell index is its LDS address),
// bitmap [max_words] (walk 5: the bitmap, then its transpose from word
// tbits_off), jobs [2E] (main, reset), pooled minima [2E][m] (+ padding), active job list [2E], misc
// [2E + 8] ([0] active jobs, [1] next ray, [2, 2 + E) done flags, [2 + E, 2 + 2E)
// reset jobs published, [2E + 6] tile vote, [2E + 7] next tile of a
// persistent workgroup), beams [K] when staged, ray slots
// [ray_cap] (none for the claim walk).
template <int E>
__device__ __forceinline__ int *fused_list(const StepParams &p) {
    extern __shared__ uint4 smem4[];
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(smem4) + p.cell_bytes);
    TileJob *s_jobs = reinterpret_cast<TileJob *>(s_bits + p.max_words);
    uint32_t *s_pool = reinterpret_cast<uint32_t *>(s_jobs + 2 * E);
    return reinterpret_cast<int *>(s_pool + pool_words(E, p.m));
}

// One tile with a workgroup of T threads (T / 64 wavefronts).
template <int E, int T>
__device__ __forceinline__ void fused_tile(const StepParams &p, int tile_index, int &staged_map) {
    extern __shared__ uint4 smem4[];
    uint8_t *s_cells = reinterpret_cast<uint8_t *>(smem4);
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(s_cells + p.cell_bytes);
    TileJob *s_jobs = reinterpret_cast<TileJob *>(s_bits + p.max_words);
    uint32_t *s_pool = reinterpret_cast<uint32_t *>(s_jobs + 2 * E);
    int *s_list = fused_list<E>(p);
    int *s_misc = s_list + 2 * E;
    double2 *s_beam = reinterpret_cast<double2 *>(s_misc + 2 * E + 8);  // [K] beams, or global
    uint4 *s_ray = reinterpret_cast<uint4 *>(s_beam + (p.beams_lds ? p.K : 0));  // [ray_cap]
    const int tid = threadIdx.x, lane = tid & 63;
    const Tile tile = p.tiles[tile_index];
    if (p.mode == 1 && p.mask) {
        // a masked reset pass: a tile with no masked env has nothing to do
        // (its envs' rows stay untouched), so it skips the map staging too.
        // The vote goes through a free word of the misc block (no static LDS:
        // the byte walk needs its map copy at address 0)
        int *s_vote = s_misc + 2 * E + 6;
        if (tid == 0) *s_vote = 0;
        __syncthreads();
        if (tid < tile.count && p.mask[p.perm[tile.first + tid]]) *s_vote = 1;
        __syncthreads();
        if (*s_vote == 0) {
            if (p.defer_out && tid < tile.count) p.defer_out[p.perm[tile.first + tid]] = 0;
            return;
        }
    }
    const MapDesc md = p.maps[tile.map];
    const int K = md.K, m = p.m, per = K / m;
    const double2 *beams = p.beams + md.beam_off;  // this map's beam directions
    // the motion's inputs (one group of 16 lanes per env), loaded before the
    // map is staged so that the two memory latencies overlap
    const int grp = tid >> 4, li = tid & 15;
    const bool mover = grp < E && grp < tile.count;
    int me = 0, mt = 0;
    uint32_t mep = 0u;
    float2 ma = make_float2(0.0f, 0.0f);
    float mx = 0.0f, my = 0.0f, mth = 0.0f, mgx = 0.0f, mgy = 0.0f, mdprev = 0.0f;
    if (mover) {
        me = p.perm[tile.first + grp];
        mep = p.st.ep[me];
        if (p.mode != 1) {
            ma = env_action(p, me);
            mx = p.st.x[me];
            my = p.st.y[me];
            mth = p.st.th[me];
            mgx = p.st.gx[me];
            mgy = p.st.gy[me];
            mdprev = p.st.dprev[me];
            mt = p.st.t[me] + 1;
        }
    }
    if (tile.map != staged_map) {  // a persistent workgroup keeps its map between tiles
        const uint4 *g = reinterpret_cast<const uint4 *>(p.bits + md.word_off);
        uint4 *b4 = reinterpret_cast<uint4 *>(s_bits);
        for (int q = tid; q < md.words / 4; q += T) b4[q] = g[q];
        if (p.tbits_off) {
            const uint4 *gt = reinterpret_cast<const uint4 *>(p.bits + md.word_off_t);
            uint4 *t4 = reinterpret_cast<uint4 *>(s_bits + p.tbits_off);
            for (int q = tid; q < md.words_t / 4; q += T) t4[q] = gt[q];
        }
        if (p.cell_bytes) {
            // byte copy: bit b of word q becomes byte 32 q + b (0 or 1); a
            // nibble times 0x00204081 moves its bit i to bit 8 i
            const uint32_t *gw = p.bits + md.word_off;
            uint4 *c4 = reinterpret_cast<uint4 *>(s_cells);
            for (int q = tid; q < md.words; q += T) {
                const uint32_t w = gw[q];
                uint32_t d[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) d[j] = (((w >> (4 * j)) & 0xFu) * 0x00204081u) & 0x01010101u;
                c4[2 * q] = make_uint4(d[0], d[1], d[2], d[3]);
                c4[2 * q + 1] = make_uint4(d[4], d[5], d[6], d[7]);
            }
        }
        if (p.beams_lds)
            for (int q = tid; q < K; q += T) s_beam[q] = beams[q];
        staged_map = tile.map;
    }
    if (!p.beams_lds) s_beam = const_cast<double2 *>(beams);
    __syncthreads();
    const MapView M = map_view(s_bits, md);
    const bool want_debug = p.d_ranges || p.d_hits || p.d_visits;

    // ---- motion: one group of 16 lanes per env ----
    bool later_reset = false;  // this group draws its env's reset pose after the job list
    int reset_env = 0;
    uint32_t reset_ep = 0u;
    if (grp < E) {
        // the rest of the workgroup waits for this: let it win issue slots from
        // other workgroups' walks on the same SIMD
        __builtin_amdgcn_s_setprio(3);
        bool active = false, done = false, defer = false;
        uint32_t ep = 0u;
        if (mover) {
            const int e = me;
            active = true;
            ep = mep;
            if (p.mode == 1) {
                done = !p.mask || p.mask[e];
                defer = done && p.defer_bin && p.defer_bin[e] >= 0;
                if (li == 0) {
                    s_jobs[grp].dst = 3;
                    if (p.defer_out) p.defer_out[e] = (uint8_t)defer;
                }
            } else {
                const float2 a = ma;
                const float x0 = mx, y0 = my, th0 = mth;
                const float gx = mgx, gy = mgy, dprev = mdprev;
                const int t = mt;
                if (p.act_out && li == 0)
                    *reinterpret_cast<float2 *>(p.act_out + 2 * (int64_t)e) = a;
                const Motion mo = apply_action(p, a.x, a.y, x0, y0, th0);
                const double x1 = (double)mo.x1, y1 = (double)mo.y1, th1 = (double)mo.th1;
                double sn, c;
                sincos(th1, &sn, &c);
                const bool coll = group_footprint_hits(M, robot_of(md), x1, y1, c, sn, li);
                double d64;
                float d32, phi;
                goal_features(x1, y1, c, sn, gx, gy, d64, d32, phi);
                const bool goal = d64 < (double)p.goal_r;
                const bool term = goal || coll;
                const bool trunc = (t >= p.horizon) && !term;
                done = term || trunc;
                defer = done && p.defer_bin && p.defer_bin[e] >= 0;
                if (li == 0) {
                    if (p.defer_out) p.defer_out[e] = (uint8_t)defer;
                    const float rew =
                        goal ? p.r_succ
                             : (coll ? p.r_coll
                                     : (float)((double)p.c1 * ((double)dprev - (double)d32)));
                    p.reward[e] = rew;
                    p.term[e] = (uint8_t)term;
                    p.trunc[e] = (uint8_t)trunc;
                    if (p.d_coll) p.d_coll[e] = (uint8_t)coll;
                    if (p.d_goal) p.d_goal[e] = (uint8_t)goal;
                    if (p.d_reset) p.d_reset[e] = (uint8_t)done;
                    if (p.d_fb) p.d_fb[e] = 0;
                    float *row = done ? p.final_obs : p.obs;
                    if (row) {
                        row += (int64_t)e * (m + 4);
                        row[m] = d32;
                        row[m + 1] = phi;
                        row[m + 2] = mo.v;
                        row[m + 3] = mo.w;
                    }
                    int dst = done ? (p.final_obs ? 1 : 2) : 0;
                    if (dst == 2 && !want_debug) dst = 3;
                    make_tile_job(s_jobs[grp], M, mo.x1, mo.y1, c, sn, e, dst);
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
            }
            if (done && !defer) {
                later_reset = true;
                reset_env = e;
                reset_ep = ep;
            }
        }
        if (li == 0) {
            if (!active) s_jobs[grp].dst = 3;
            s_misc[2 + grp] = (active && done && !defer) ? 1 : 0;
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    if (tid < 64) {
        // active jobs in order (main jobs 0..E-1, then resets E..2E-1): lane q
        // tests job q, a ballot and a prefix count give its list position
        const bool on = tid < E ? s_jobs[tid].dst != 3 : (tid < 2 * E && s_misc[2 + tid - E] != 0);
        const uint64_t bm = __ballot(on);
        if (on) s_list[__popcll(bm & ((1ull << tid) - 1ull))] = tid;
        if (tid < E) s_misc[2 + E + tid] = 0;  // reset jobs not yet published
        if (tid == 0) {
            s_misc[0] = __popcll(bm);
            s_misc[1] = 0;
        }
    }
    for (int q = tid; q < 2 * E * m; q += T) s_pool[q] = 0x7f800000u;  // +inf
    __syncthreads();
    if (later_reset) {
        // a done env's reset pose, drawn by its group of 16 lanes; in the claim
        // walks the other wavefronts start walking meanwhile (see wait_job_ready)
        __builtin_amdgcn_s_setprio(3);
        double c = 1.0, sn = 0.0;
        ResetPose r;
        if (p.pose && (!p.pose_src || p.pose_src[reset_env] >= 0)) {
            r = given_pose(p, reset_env);
            sincos((double)r.th, &sn, &c);
        } else {
            r = group_sample_reset(p, M, md, reset_env, reset_ep, li, c, sn);
        }
        if (li == 0) {
            store_reset_cs(p, reset_env, reset_ep, r, c, sn);
            make_tile_job(s_jobs[E + grp], M, r.x, r.y, c, sn, reset_env, 0);
            __hip_atomic_store(s_misc + 2 + E + grp, 1, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (!p.claim) __syncthreads();  // the chunked walks set up every ray at once

    // ---- scan, in chunks of at most ray_cap rays ----
    const int nj = s_misc[0];
    const int R = nj * K;
    const float inv_K = 1.0f / (float)K, inv_per = 1.0f / (float)per;
    const double rmax_c = walk_cells((double)p.rmax, M.s);
    const int max_n = M.w + M.h + 2 * kPad;  // a walk meets the padding ring before this
    if (p.claim) {
        // s_misc[1] (next ray) and the pool were cleared before the last barrier
        if (p.tbits_off)
            claim_run_walk(p, M, s_bits, s_jobs, s_list, s_beam, s_pool, s_misc, R,
                           K, inv_K, per, inv_per, rmax_c, max_n, E, lane);
        else if (p.cell_bytes)
            claim_walk<true>(p, M, s_bits, s_cells, s_jobs, s_list, s_beam, s_pool, s_misc, R, K,
                             inv_K, per, inv_per, rmax_c, max_n, E, lane);
        else
            claim_walk<false>(p, M, s_bits, s_cells, s_jobs, s_list, s_beam, s_pool, s_misc, R,
                              K, inv_K, per, inv_per, rmax_c, max_n, E, lane);
        __syncthreads();
    }
    for (int c0 = 0; c0 < R && !p.claim; c0 += p.ray_cap) {
        const int Rc = min(p.ray_cap, R - c0);
        // (1) every ray's walk start, all lanes busy (the march needs none)
        for (int r = tid; r < Rc && p.scan_mode != 1; r += T) {
            const int g = c0 + r;
            int beam;
            const int jl = small_divmod(g, K, inv_K, beam);
            const TileJob &j = s_jobs[s_list[jl]];
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (!j.blocked) {
                const double2 cs = s_beam[beam];
                const double dx = j.c * cs.x - j.s * cs.y;
                const double dy = j.s * cs.x + j.c * cs.y;
                v = pack_walk(walk_setup(M.pitch, tile_origin(j, M.s), dx, dy, rmax_c), max_n);
            }
            s_ray[r] = v;
        }
        if (tid == 0) s_misc[1] = 0;
        __syncthreads();
        // (2) walk: lanes take rays from s_misc[1]; a lane whose ray is done
        // writes its result back and takes a new one once at most refill_at
        // lanes of its wavefront are still walking
        if (p.scan_mode == 1) {
            march_walk(p, M, s_jobs, s_list, s_beam, s_ray, s_misc, c0, Rc, K, inv_K, lane);
        } else if (p.walk_mode == 1) {
            run_walk(p, M, s_bits, s_ray, s_misc, Rc, lane);
        } else if (p.walk_mode == 2) {
            group_walk<true>(p, M, s_bits, s_cells, s_ray, s_misc, Rc, lane);
        } else {
            group_walk<false>(p, M, s_bits, s_cells, s_ray, s_misc, Rc, lane);
        }
        __syncthreads();
        // (3) ranges, hits, pooling, all lanes busy
        for (int q = tid; q < Rc; q += T) {
            const int g = c0 + q;
            int beam;
            const int jl = small_divmod(g, K, inv_K, beam);
            const int job = s_list[jl];
            const uint4 v = s_ray[q];
            if (p.scan_mode == 1)
                finish_march(p, M, s_jobs[job], s_beam, job, beam, v.x, s_pool, per, inv_per, E);
            else
                finish_ray(p, M, s_jobs[job], s_beam, job, beam, make_uint2(v.x, v.y), s_pool,
                           per, inv_per, E);
        }
        __syncthreads();
    }

    // ---- pooled sector minima -> observation rows ----
    for (int q = tid; q < nj * m; q += T) {
        const int jl = q / m, sec = q - jl * m;
        const TileJob &j = s_jobs[s_list[jl]];
        float *dst = j.dst == 0 ? p.obs : (j.dst == 1 ? p.final_obs : nullptr);
        if (dst) dst[(int64_t)j.env * (m + 4) + sec] = __uint_as_float(s_pool[s_list[jl] * m + sec]);
    }
}

// One workgroup per tile (Q false), or persistent workgroups (Q true) that
// take `chunk` consecutive tiles at a time from a device counter; the last
// workgroup to finish sets the counter back to zero for the next launch.  The
// two are separate kernels: with the tile loop in the same kernel the
// compiler hoisted the math library's polynomial coefficients out of it and
// kept them in scratch memory, reloading one per step of every atan2.
// Register budget: 128 VGPRs, so that 4 wavefronts share each SIMD and hide
// one another's LDS latency in the walk (the compiler's own choice, ~200,
// leaves 2); the walk loop keeps everything in registers.
template <int E, int T, bool Q>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(kFusedWavesPerSimd)))
void fused_step_kernel(StepParams p) {
    int staged = -1;
    if constexpr (!Q) {
        fused_tile<E, T>(p, (int)blockIdx.x, staged);
        return;
    }
    int *s_next = fused_list<E>(p) + 4 * E + 7;
    for (;;) {
        if (threadIdx.x == 0) *s_next = atomicAdd(&p.queue[0], p.chunk);
        __syncthreads();
        const int t0 = *s_next;
        __syncthreads();
        if (t0 >= p.num_tiles) break;
        const int t1 = min(t0 + p.chunk, p.num_tiles);
        for (int t = t0; t < t1; ++t) {
            fused_tile<E, T>(p, t, staged);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&p.queue[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&p.queue[0], 0);
            atomicExch(&p.queue[1], 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Plain mapping: one thread per env, the whole step in sequence.

__device__ void observe_serial(const StepParams &p, const MapView &M, const MapDesc &md, double x,
                               double y, double c, double sn, float *obs_row, int64_t dbg_row) {
    const RayOrigin o = ray_origin(M, x, y);
    const double rmax = (double)p.rmax, rmax_c = walk_cells(rmax, M.s);
    const double2 *beams = p.beams + md.beam_off;
    const int per = md.K / p.m;
    for (int j = 0; j < p.m; ++j) {
        float l = 0.0f;
        for (int q = 0; q < per; ++q) {
            const int k = j * per + q;
            float rg;
            int hit, vis;
            if (p.scan_mode == 1) {
                const double2 cs = beams[k];
                const double dx = c * cs.x - sn * cs.y;
                const double dy = sn * cs.x + c * cs.y;
                march_ray(p, M, x, y, dx, dy, rg, hit, vis);
            } else if (o.blocked) {
                rg = 0.0f;
                hit = o.block_hit;
                vis = 1;
            } else {
                const double2 cs = beams[k];
                const double dx = c * cs.x - sn * cs.y;
                const double dy = sn * cs.x + c * cs.y;
                cast_ray(M, o, dx, dy, rmax, rmax_c, rg, hit, vis);
            }
            l = q == 0 ? rg : fminf(l, rg);
            if (dbg_row >= 0) {
                if (p.d_ranges) p.d_ranges[dbg_row * p.K + k] = rg;
                if (p.d_hits) p.d_hits[dbg_row * p.K + k] = hit;
                if (p.d_visits) p.d_visits[dbg_row * p.K + k] = vis;
            }
        }
        if (obs_row) obs_row[j] = l;
    }
}

__global__ __launch_bounds__(64) void plain_step_kernel(StepParams p) {
    const int e = blockIdx.x * 64 + threadIdx.x;
    if (e >= p.N) return;
    const MapDesc md = p.maps[p.env_map[e]];
    const MapView M = map_view(p.bits + md.word_off, md);
    const int row = p.m + 4;
    float *obs_row = p.obs + (int64_t)e * row;
    bool do_reset;
    if (p.mode == 1) {
        do_reset = !p.mask || p.mask[e];
    } else {
        const float2 a = env_action(p, e);
        if (p.act_out) *reinterpret_cast<float2 *>(p.act_out + 2 * (int64_t)e) = a;
        const Motion mo = apply_action(p, a.x, a.y, p.st.x[e], p.st.y[e], p.st.th[e]);
        const double x1 = (double)mo.x1, y1 = (double)mo.y1, th1 = (double)mo.th1;
        const bool coll = footprint_hits(M, robot_of(md), x1, y1, th1);
        double sn, c;
        sincos(th1, &sn, &c);
        double d64;
        float d32, phi;
        goal_features(x1, y1, c, sn, p.st.gx[e], p.st.gy[e], d64, d32, phi);
        const bool goal = d64 < (double)p.goal_r;
        const int t = p.st.t[e] + 1;
        const bool term = goal || coll;
        const bool trunc = (t >= p.horizon) && !term;
        do_reset = term || trunc;
        const float rew =
            goal ? p.r_succ
                 : (coll ? p.r_coll : (float)((double)p.c1 * ((double)p.st.dprev[e] - (double)d32)));
        float *pre = do_reset ? (p.final_obs ? p.final_obs + (int64_t)e * row : nullptr) : obs_row;
        observe_serial(p, M, md, x1, y1, c, sn, pre, e);
        if (pre) {
            pre[p.m] = d32;
            pre[p.m + 1] = phi;
            pre[p.m + 2] = mo.v;
            pre[p.m + 3] = mo.w;
        }
        p.reward[e] = rew;
        p.term[e] = (uint8_t)term;
        p.trunc[e] = (uint8_t)trunc;
        if (p.d_coll) p.d_coll[e] = (uint8_t)coll;
        if (p.d_goal) p.d_goal[e] = (uint8_t)goal;
        if (p.d_reset) p.d_reset[e] = (uint8_t)do_reset;
        if (p.d_fb) p.d_fb[e] = 0;
        if (!do_reset) {
            p.st.x[e] = mo.x1;
            p.st.y[e] = mo.y1;
            p.st.th[e] = mo.th1;
            p.st.v[e] = mo.v;
            p.st.w[e] = mo.w;
            p.st.dprev[e] = d32;
            p.st.t[e] = t;
        }
    }
    if (!do_reset) return;
    const uint32_t ep = p.st.ep[e];
    const ResetPose r = (p.pose && (!p.pose_src || p.pose_src[e] >= 0))
                            ? given_pose(p, e)
                            : sample_reset(p, M, md, e, ep);
    double c, sn;
    store_reset(p, e, ep, r, c, sn);
    observe_serial(p, M, md, (double)r.x, (double)r.y, c, sn, obs_row, -1);
}

// ---------------------------------------------------------------------------
template <int E, int T, bool Q>
static hipError_t launch_fused_etq(const StepParams &p, hipStream_t s) {
    const size_t lds = fused_lds_bytes(p.max_words, p.m, E, p.beams_lds ? p.K : 0,
                                       p.claim ? 0 : p.ray_cap, p.cell_bytes);
    if (lds > 65536u) {
        // dynamic LDS beyond 64 KiB (gfx950 allows up to 160 KiB per workgroup),
        // raised once per device and size
        constexpr int kDevices = 64;
        static std::atomic<int> raised[kDevices];
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kDevices || (int)lds > raised[dev].load()) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(fused_step_kernel<E, T, Q>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            if (dev >= 0 && dev < kDevices) raised[dev].store((int)lds);
        }
    }
    unsigned grid = (unsigned)p.num_tiles;
    if (p.queue) {
        // at most the resident workgroups, and one per chunk of tiles
        const int chunks = (p.num_tiles + p.chunk - 1) / p.chunk;
        grid = (unsigned)std::max(1, std::min(chunks, p.resident));
    }
    hipLaunchKernelGGL((fused_step_kernel<E, T, Q>), dim3(grid), dim3(T), lds, s, p);
    return hipGetLastError();
}

template <int E, int T>
static hipError_t launch_fused_et(const StepParams &p, hipStream_t s) {
    return p.queue ? launch_fused_etq<E, T, true>(p, s) : launch_fused_etq<E, T, false>(p, s);
}

template <int E, int T>
static int resident_et(size_t lds) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_step_kernel<E, T, false>, T,
                                                     lds) !=
            hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

// Every supported (tile_envs, threads) pair.
// (32-env tiles need 16 lanes per env in the motion phase: 512 threads or more)
#define NAVSIM_FUSED_SHAPES(X)                                                                \
    X(1, 256) X(1, 512) X(1, 1024) X(2, 256) X(2, 512) X(2, 1024) X(4, 256) X(4, 512)        \
    X(4, 1024) X(8, 256) X(8, 512) X(8, 1024) X(16, 256) X(16, 512) X(16, 1024) X(32, 512)   \
    X(32, 1024)

int fused_resident_groups(int max_words, int m, int E, int T, int K, bool beams_lds, int ray_cap,
                          int cell_bytes) {
    const size_t lds = fused_lds_bytes(max_words, m, E, beams_lds ? K : 0, ray_cap, cell_bytes);
#define NAVSIM_X(e, t) \
    if (E == e && T == t) return resident_et<e, t>(lds);
    NAVSIM_FUSED_SHAPES(NAVSIM_X)
#undef NAVSIM_X
    return 0;
}

template <int E, int T>
static int static_lds_et() {
    hipFuncAttributes fa, fq;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(fused_step_kernel<E, T, false>)) !=
            hipSuccess ||
        hipFuncGetAttributes(&fq, reinterpret_cast<const void *>(fused_step_kernel<E, T, true>)) !=
            hipSuccess)
        return -1;
    return (int)std::max(fa.sharedSizeBytes, fq.sharedSizeBytes);
}

int fused_static_lds(int E, int T) {
#define NAVSIM_X(e, t) \
    if (E == e && T == t) return static_lds_et<e, t>();
    NAVSIM_FUSED_SHAPES(NAVSIM_X)
#undef NAVSIM_X
    return -1;
}

bool fused_tile_envs_supported(int E) {
    return E == 1 || E == 2 || E == 4 || E == 8 || E == 16 || E == 32;
}
bool fused_threads_supported(int T) { return T == 256 || T == 512 || T == 1024; }

// LDS walk slots per chunk: the rays of a full tile plus one reset pose
// ((E + 1) K, rounded up to a wavefront), so a tile walks a second chunk only
// when two or more of its envs reset; fewer if that does not fit `budget`
// bytes of LDS; 0 if not even 256 do.
int fused_ray_cap(int max_words, int m, int E, int K, bool beams_lds, int budget, int cell_bytes) {
    const size_t base = fused_lds_bytes(max_words, m, E, beams_lds ? K : 0, 0, cell_bytes);
    if (base + 16u * 256u > (size_t)budget) return 0;
    const int fit = (int)(((size_t)budget - base) / 16u) & ~63;
    return std::max(std::min(((E + 1) * K + 63) & ~63, fit), 256);
}

hipError_t launch_fused(const StepParams &p, int tile_envs, hipStream_t s) {
    if (p.num_tiles == 0) return hipSuccess;
#define NAVSIM_X(e, t) \
    if (tile_envs == e && p.wg_threads == t) return launch_fused_et<e, t>(p, s);
    NAVSIM_FUSED_SHAPES(NAVSIM_X)
#undef NAVSIM_X
    return hipErrorInvalidValue;
}

// Sets the rollout's first step index in device memory, so that a captured
// sequence of steps can be replayed for any index.
__global__ void set_step_kernel(uint32_t *ctr, uint32_t lo, uint32_t hi) {
    if (threadIdx.x == 0) {
        ctr[0] = lo;
        ctr[1] = hi;
    }
}

hipError_t launch_set_step(uint32_t *ctr, uint64_t first_step, hipStream_t s) {
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, s, ctr, (uint32_t)first_step,
                       (uint32_t)(first_step >> 32));
    return hipGetLastError();
}

hipError_t launch_plain(const StepParams &p, hipStream_t s) {
    const unsigned blocks = (unsigned)((p.N + 63) / 64);
    hipLaunchKernelGGL(plain_step_kernel, dim3(blocks), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace navsim
