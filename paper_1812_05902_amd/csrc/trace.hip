// The per-ray pipeline of sec. 3 in one kernel: emit (3.1) -> integrate through the index grid
// (3.2, eqs. 3-6) -> aperture and thick lens (3.3, eq. 7) -> sensor hit and erf-integrated
// Gaussian spot (3.4, eq. 8), deposited as Q32.32 integers with 64-bit atomics.
//
// Precision layout.  The integration inside the box runs in the template type F (float by
// default).  Positions are kept cell-local: an integer cell index plus a fraction of the cell
// (summed in FP64, see rkn_step), so the rounding of a position is relative to the cell size
// rather than to the metres of the scene.  The direction vector T = n dR/ds is kept as its value at the box entry (T_ref,
// constant) plus the accumulated change dT, so the small increments (A + 4B + C)/6 are summed
// into a small number.  Emission, the box entry, the lens and the sensor run in FP64: they cost a
// few hundred operations per ray against a few hundred thousand in the integration loop.
#include "pbr_internal.h"

namespace pbr {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kTwoPow32 = 4294967296.0;

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) evaluated at counter k: output number k of the
// generator seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Checked builds: the access that the caller is about to make is in range if ok; a failed test
// is counted in the CNT_BAD_ACCESS slot, and the caller then clamps the index into its buffer or
// skips the access.  Regular builds return true and compile the test and its fix-up out.
__device__ __forceinline__ bool access_ok(const TraceParams &P, bool ok)
{
#if PBR_CHECKED
    if (!ok && P.counters)
        __hip_atomic_fetch_add(P.counters + CNT_BAD_ACCESS, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ok;
#else
    (void)P;
    (void)ok;
    return true;
#endif
}

// x clamped to [0, hi] in one instruction (for a bound that is not a constant the compiler emits a
// max and a min); hi is uniform across the wave.
__device__ __forceinline__ int clamp_index(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// A stage-point coordinate x (cell units, relative to the ray's cell) split into the whole cells it
// lies ahead, floor(x), and the fraction x - floor(x) inside that cell.  For float two instructions
// (v_cvt_flr_i32_f32 saturates out-of-range values; v_fract_f32 keeps the fraction below 1).
template <typename F> __device__ __forceinline__ int split_cell(F x, F &t);
template <> __device__ __forceinline__ int split_cell<float>(float x, float &t)
{
    int o;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(o) : "v"(x));
    t = __builtin_amdgcn_fractf(x);
    return o;
}
template <> __device__ __forceinline__ int split_cell<double>(double x, double &t)
{
    const double o = floor(x);
    t = x - o;
    return (int)o;
}

// The coefficients (cell layout) or corner values (node layout) of the cell the ray is in, held
// in registers: a stage point only gathers
// from memory when it lies in another cell (about once per cell crossing, since the three stage
// points of a step run ahead of the ray).
struct CellCache {
    int ix, iy, iz;  // the cached cell, ix = -1: none
    float4 c[kCellFloat4];
};

// Node layout: the eight corners (n - 1, grad n) of cell ic, in the order 000, 100, 010, 001, 110,
// 101, 011, 111 (x, y, z offsets), loaded into the cache.  They are interpolated as they are (see
// sample_field): steps in the fine grids this layout serves cross a cell every one or two
// samples, so a per-gather transform into polynomial coefficients would cost more than it saves.
// A move to a face neighbour of the cached cell keeps the four corners of the shared face and
// loads the other four: half the gather traffic on most crossings.
__device__ __forceinline__ void gather_nodes(const TraceParams &P, const int ic[3], CellCache &cc)
{
    const size_t sy = (size_t)P.nx, sz = (size_t)P.nx * (size_t)P.ny;
    {   // Every gathering lane wants the same cell (about a quarter of the gathers on the Tomo-PIV
        // image, a wave's rays travelling together): its eight corners through the scalar cache,
        // which takes them off the texture-data path, the bound of this kernel on fine grids.
        const int u0 = __builtin_amdgcn_readfirstlane(ic[0]), u1 = __builtin_amdgcn_readfirstlane(ic[1]),
                  u2 = __builtin_amdgcn_readfirstlane(ic[2]);
        const bool same = (ic[0] == u0) & (ic[1] == u1) & (ic[2] == u2);
        if (__builtin_amdgcn_ballot_w64(!same) == 0ull) {
            typedef __attribute__((address_space(4))) const float cfloat;  // constant: scalar loads
            cfloat *s = (cfloat *)(P.cells + (size_t)u2 * sz + (size_t)u1 * sy + (size_t)u0);
            auto at = [&](size_t o) { return make_float4(s[4 * o], s[4 * o + 1], s[4 * o + 2], s[4 * o + 3]); };
            float4 *c = cc.c;
            c[0] = at(0); c[1] = at(1); c[2] = at(sy); c[3] = at(sz);
            c[4] = at(sy + 1); c[5] = at(sz + 1); c[6] = at(sz + sy); c[7] = at(sz + sy + 1);
            return;
        }
    }
    const float4 *b = P.cells + (size_t)ic[2] * sz + (size_t)ic[1] * sy + (size_t)ic[0];
    float4 *c = cc.c;
    const int dx = ic[0] - cc.ix, dy = ic[1] - cc.iy, dz = ic[2] - cc.iz;
    const bool one = cc.ix >= 0 && abs(dx) + abs(dy) + abs(dz) == 1;  // ix = -1: nothing cached
    if (one && dz == 1) {
        c[0] = c[3]; c[1] = c[5]; c[2] = c[6]; c[4] = c[7];
        c[3] = b[sz]; c[5] = b[sz + 1]; c[6] = b[sz + sy]; c[7] = b[sz + sy + 1];
    } else if (one && dz == -1) {
        c[3] = c[0]; c[5] = c[1]; c[6] = c[2]; c[7] = c[4];
        c[0] = b[0]; c[1] = b[1]; c[2] = b[sy]; c[4] = b[sy + 1];
    } else if (one && dx == 1) {
        c[0] = c[1]; c[2] = c[4]; c[3] = c[5]; c[6] = c[7];
        c[1] = b[1]; c[4] = b[sy + 1]; c[5] = b[sz + 1]; c[7] = b[sz + sy + 1];
    } else if (one && dx == -1) {
        c[1] = c[0]; c[4] = c[2]; c[5] = c[3]; c[7] = c[6];
        c[0] = b[0]; c[2] = b[sy]; c[3] = b[sz]; c[6] = b[sz + sy];
    } else if (one && dy == 1) {
        c[0] = c[2]; c[1] = c[4]; c[3] = c[6]; c[5] = c[7];
        c[2] = b[sy]; c[4] = b[sy + 1]; c[6] = b[sz + sy]; c[7] = b[sz + sy + 1];
    } else if (one && dy == -1) {
        c[2] = c[0]; c[4] = c[1]; c[6] = c[3]; c[7] = c[5];
        c[0] = b[0]; c[1] = b[1]; c[3] = b[sz]; c[5] = b[sz + 1];
    } else {
        c[0] = b[0]; c[1] = b[1]; c[2] = b[sy]; c[3] = b[sz];
        c[4] = b[sy + 1]; c[5] = b[sz + 1]; c[6] = b[sz + sy]; c[7] = b[sz + sy + 1];
    }
}

// The same gather with every load issued last: the kept corners are shifted one axis at a time
// (z, then x, then y, so a diagonal move keeps what it can), and each corner the new cell still
// lacks is loaded by one instruction masked to the lanes that lack it.  The cache ends up with the
// same eight values.  It issues 37% fewer load instructions on the Tomo-PIV image but moves the
// same bytes, which is what the texture-data path spends its time on, and costs more vector and
// scalar instructions; what it does save is registers, so the kernels that also hold FP64 steps
// (mixed precision, calibration) use it: four waves per SIMD instead of three.
__device__ __forceinline__ void gather_nodes_deferred(const TraceParams &P, const int ic[3], CellCache &cc)
{
    const size_t sy = (size_t)P.nx, sz = (size_t)P.nx * (size_t)P.ny;
    const float4 *b = P.cells + (size_t)ic[2] * sz + (size_t)ic[1] * sy + (size_t)ic[0];
    float4 *c = cc.c;
    const int dx = ic[0] - cc.ix, dy = ic[1] - cc.iy, dz = ic[2] - cc.iz;
    const bool near = cc.ix >= 0 && (unsigned)(dx + 1) <= 2u && (unsigned)(dy + 1) <= 2u && (unsigned)(dz + 1) <= 2u;
    // corners of the new cell that the cached cell does not hold: slot bits of the x = 1 corners
    // (1, 4, 5, 7), the x = 0 corners (0, 2, 3, 6), likewise for y and z
    unsigned need = 0xFFu;
    if (near) {
        need = (dx == 1 ? 0xB2u : dx == -1 ? 0x4Du : 0u) | (dy == 1 ? 0xD4u : dy == -1 ? 0x2Bu : 0u) |
               (dz == 1 ? 0xE8u : dz == -1 ? 0x17u : 0u);
        // shift the kept corners into place, one axis at a time (register copies only: every load
        // is issued at the end, so no copy waits on one)
        if (dz == 1) {
            c[0] = c[3]; c[1] = c[5]; c[2] = c[6]; c[4] = c[7];
            asm volatile("");  // keeps mirrored branches apart (no merged stores through selected addresses)
        } else if (dz == -1) {
            c[3] = c[0]; c[5] = c[1]; c[6] = c[2]; c[7] = c[4];
        }
        if (dx == 1) {
            c[0] = c[1]; c[2] = c[4]; c[3] = c[5]; c[6] = c[7];
            asm volatile("");
        } else if (dx == -1) {
            c[1] = c[0]; c[4] = c[2]; c[5] = c[3]; c[7] = c[6];
        }
        if (dy == 1) {
            c[0] = c[2]; c[1] = c[4]; c[3] = c[6]; c[5] = c[7];
            asm volatile("");
        } else if (dy == -1) {
            c[2] = c[0]; c[4] = c[1]; c[6] = c[3]; c[7] = c[5];
        }
    }
    if (need & 0x01u) c[0] = b[0];
    if (need & 0x02u) c[1] = b[1];
    if (need & 0x04u) c[2] = b[sy];
    if (need & 0x08u) c[3] = b[sz];
    if (need & 0x10u) c[4] = b[sy + 1];
    if (need & 0x20u) c[5] = b[sz + 1];
    if (need & 0x40u) c[6] = b[sz + sy];
    if (need & 0x80u) c[7] = b[sz + sy + 1];
}

// Trilinear interpolation of (n - 1, grad n) at the point (cell c, fraction f); the fraction may
// lie outside [0, 1) (stage points of eq. 5), in which case the point is moved into the cell that
// holds it and then onto the box.  Returns n, writes G = grad n (D = n G, eq. 6, is formed by the
// caller, folded into the step's sums).
// INSIDE: the caller has shown that the point lies inside the box and that the ray's own cell index
// is a cell of the grid (see trace_step), so the edge extension is left out; a stage point's cell
// index is still clamped to the grid, which keeps every gather in bounds whatever the values.
// NODES: the field is stored per node (see gather_nodes); compiled into dedicated kernels only.
template <typename F, bool AT_STATE = false, bool INSIDE = false, int NODES = 0>
__device__ __forceinline__ F sample_field(const TraceParams &P, CellCache &cc, const int c[3],
                                          const F f[3], F G[3])
{
    const int nmax[3] = {P.nx - 2, P.ny - 2, P.nz - 2};
    int ic[3];
    F w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int i0;
        F t;
        if (AT_STATE) {
            // the ray's own position: fraction already in [0, 1], cell normally valid
            i0 = c[a];
            t = f[a];
        } else {
            // stage point: fraction anywhere.  Inside the box the point is finite (see trace_step);
            // elsewhere NaN becomes finite first (fmax/fmin return the number)
            const F fa = INSIDE ? f[a] : fmin(fmax(f[a], (F)(-1.0e6)), (F)(1.0e6));
            i0 = c[a] + split_cell<F>(fa, t);
        }
        // (every step starts in a cell of the grid, so an inside step's own index needs no clamp)
        const int i = INSIDE ? (AT_STATE ? i0 : clamp_index(i0, nmax[a])) : min(max(i0, 0), nmax[a]);
        if (!INSIDE) {
            t = i0 < 0 ? (F)0 : t;
            t = i0 > nmax[a] ? (F)1 : t;
        }
        ic[a] = i;
        w[a] = t;
    }
    // compare cell coordinates (no index arithmetic unless the cell changed)
    if ((ic[0] != cc.ix) | (ic[1] != cc.iy) | (ic[2] != cc.iz)) {
        if (PBR_CHECKED && !access_ok(P, (unsigned)ic[0] <= (unsigned)nmax[0] && (unsigned)ic[1] <= (unsigned)nmax[1] &&
                                             (unsigned)ic[2] <= (unsigned)nmax[2])) {
#pragma unroll
            for (int a = 0; a < 3; ++a) ic[a] = min(max(ic[a], 0), nmax[a]);
        }
        if (NODES == 2) gather_nodes_deferred(P, ic, cc);
        else if (NODES) gather_nodes(P, ic, cc);
        else {
            const int key = (ic[2] * (P.ny - 1) + ic[1]) * (P.nx - 1) + ic[0];
            const float4 *p = P.cells + (size_t)key * kCellFloat4;
#pragma unroll
            for (int m = 0; m < kCellFloat4; ++m) cc.c[m] = p[m];
        }
        cc.ix = ic[0];
        cc.iy = ic[1];
        cc.iz = ic[2];
    }
    const F x = w[0], y = w[1], z = w[2];
    F v[4];
    if (NODES) {
        // seven linear interpolations per quantity from the corners: along x on the four edges,
        // then y, then z
#define PBR_LERP(a, b, t) ((a) + (t) * ((b) - (a)))
#define PBR_TRI(ch, out)                                                                   \
    {                                                                                      \
        const F e00 = PBR_LERP((F)cc.c[0].ch, (F)cc.c[1].ch, x);                           \
        const F e10 = PBR_LERP((F)cc.c[2].ch, (F)cc.c[4].ch, x);                           \
        const F e01 = PBR_LERP((F)cc.c[3].ch, (F)cc.c[5].ch, x);                           \
        const F e11 = PBR_LERP((F)cc.c[6].ch, (F)cc.c[7].ch, x);                           \
        out = PBR_LERP(PBR_LERP(e00, e10, y), PBR_LERP(e01, e11, y), z);                   \
    }
        PBR_TRI(x, v[0]);
        PBR_TRI(y, v[1]);
        PBR_TRI(z, v[2]);
        PBR_TRI(w, v[3]);
#undef PBR_TRI
#undef PBR_LERP
    } else {
        // the cell's polynomial c0 + x c1 + y c2 + z c3 + xy c4 + xz c5 + yz c6 + xyz c7, Horner form
#define PBR_TRI(ch, out)                                                                   \
    {                                                                                      \
        const F t1 = (F)cc.c[4].ch + z * (F)cc.c[7].ch;                                    \
        const F t2 = (F)cc.c[1].ch + y * t1 + z * (F)cc.c[5].ch;                           \
        const F t3 = (F)cc.c[2].ch + z * (F)cc.c[6].ch;                                    \
        out = (F)cc.c[0].ch + z * (F)cc.c[3].ch + y * t3 + x * t2;                         \
    }
        PBR_TRI(x, v[0]);
        PBR_TRI(y, v[1]);
        PBR_TRI(z, v[2]);
        PBR_TRI(w, v[3]);
#undef PBR_TRI
    }
    G[0] = v[1];
    G[1] = v[2];
    G[2] = v[3];
    return (F)1 + v[0];
}

// Margin (cells) that a full step taken without the edge extension keeps from every face.
constexpr float kFaceMargin = 1.0e-3f;

// Per-launch constants of the integration loop.
template <typename F> struct StepGeom {
    F g[3], gh[3];     // h / spacing (cell units per unit of T in a full step), half of it
    F hstep, h4, h2, h6;  // h, h / 4, h / 2, h * (1/6)
    int last[3];       // n - 1 per axis (the upper face, in cells)
    int lo[3];         // interior margin k: cells a full step may cross
    unsigned bnd[3];   // max(n - 1 - 2k, 0): interior cells are k <= c < k + bnd
    F tlim;            // largest |T| component for which a full step crosses fewer than k - 4 kFaceMargin cells
};

template <typename F> __device__ __forceinline__ StepGeom<F> step_geom(const TraceParams &P);
// FP32: the constants the host rounded once (uniform: scalar registers)
template <> __device__ __forceinline__ StepGeom<float> step_geom<float>(const TraceParams &P)
{
    StepGeom<float> s;
    const int nn[3] = {P.nx, P.ny, P.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.g[a] = P.g32[a];
        s.gh[a] = P.gh32[a];
        s.last[a] = nn[a] - 1;
        s.lo[a] = P.kin[a];
        s.bnd[a] = (unsigned)max(nn[a] - 1 - 2 * P.kin[a], 0);
    }
    s.hstep = P.h32;
    s.h4 = P.h4_32;
    s.h2 = P.h2_32;
    s.h6 = P.h6_32;
    s.tlim = P.tlim32;
    return s;
}
template <> __device__ __forceinline__ StepGeom<double> step_geom<double>(const TraceParams &P)
{
    StepGeom<double> s;
    const int nn[3] = {P.nx, P.ny, P.nz};
    s.tlim = 3.0e38;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.g[a] = P.step_cell[a];
        s.gh[a] = 0.5 * s.g[a];
        s.last[a] = nn[a] - 1;
        s.lo[a] = P.kin[a];
        s.bnd[a] = (unsigned)max(nn[a] - 1 - 2 * P.kin[a], 0);
        s.tlim = fmin(s.tlim, ((double)P.kin[a] - 4.0 * (double)kFaceMargin) / s.g[a]);
    }
    s.hstep = P.h;
    s.h4 = 0.25 * P.h;
    s.h2 = 0.5 * P.h;
    s.h6 = P.h * (1.0 / 6.0);
    return s;
}

// One step of eqs. 3 and 5 of length lam * h in the parameter t (dR/dt = T, dT/dt = D), in
// cell units: g[a] = h / spacing[a].  The cell fraction fd is accumulated in FP64: its increment
// is nearly the same every step, so FP32 rounding of the running sum would err the same way
// every step and grow linearly with the step count.  Stage points are formed in F.
// With D_A, D_B, D_C the values of D = n grad n at the three stage points, so that eq. 5's
// A = h D_A, B = h D_B, C = h D_C, the sums are regrouped without forming A, B, C:
//   stage B point  R + (h/2) (T + (h/4) D_A)        (= R + h (T/2 + A/8))
//   stage C point  R + h (T + (h/2) D_B)            (= R + h (T + B/2))
//   R'             R + h (T + (h/6) (D_A + 2 D_B))  (= R + h (T + (A + 2B)/6))
//   T'             T + (h/6) (D_A + 4 D_B + D_C)    (= T + (A + 4B + C)/6)
// A partial step (lam = 1) and a full step form the same constants and give the same bits.
// INSIDE: every point of the step is known to lie inside the box (full steps only).
template <typename F, bool FULL, bool INSIDE = false, int NODES = 0>
__device__ __forceinline__ void rkn_step(const TraceParams &P, CellCache &cc, int c[3], double fd[3],
                                         const F Tr[3], F dT[3], const StepGeom<F> &sg, F lam)
{
    const F hh = FULL ? sg.hstep : lam * sg.hstep;
    const F h4 = FULL ? sg.h4 : (F)0.25 * hh, h2 = FULL ? sg.h2 : (F)0.5 * hh;
    const F h6 = FULL ? sg.h6 : hh * ((F)1 / (F)6);
    F f[3], gg[3], gh[3], T[3], G[3], q[3], DA[3], DB[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[a] = (F)fd[a];
        gg[a] = FULL ? sg.g[a] : lam * sg.g[a];
        gh[a] = FULL ? sg.gh[a] : (F)0.5 * gg[a];
        T[a] = Tr[a] + dT[a];
    }
    F n = sample_field<F, true, INSIDE, NODES>(P, cc, c, f, G);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        DA[a] = n * G[a];
        q[a] = f[a] + gh[a] * (T[a] + h4 * DA[a]);
    }
    n = sample_field<F, false, INSIDE, NODES>(P, cc, c, q, G);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        DB[a] = n * G[a];
        q[a] = f[a] + gg[a] * (T[a] + h2 * DB[a]);
    }
    n = sample_field<F, false, INSIDE, NODES>(P, cc, c, q, G);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fd[a] += (double)(gg[a] * (T[a] + h6 * (DA[a] + (F)2 * DB[a])));
        dT[a] = dT[a] + h6 * (n * G[a] + (DA[a] + (F)4 * DB[a]));
        const double o = floor(fd[a]);
        c[a] += (int)o;
        fd[a] -= o;
    }
}

template <typename T> __device__ __forceinline__ T pick3(const T v[3], int k)
{
    return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
}

// Exit rule: before each step find the smallest straight-line step fraction lam at which the ray
// reaches a face it moves towards; if lam <= 1 take one step of lam (when lam > 0), then move
// straight along the new T onto that face.  (Per-axis values are selected with pick3 / unrolled
// loops: no dynamically indexed arrays.)
enum : int { STEP_GO = 0, STEP_EXIT = 1, STEP_LIMIT = 2 };

// One iteration of the integration: a full step, or (when the straight line of a full step reaches
// a face the ray moves towards) the partial step of fraction lam and, if the ray still heads out,
// the straight move onto that face.  Returns STEP_EXIT when the ray left the box, STEP_LIMIT when
// it ran out of steps, STEP_GO otherwise.
// A full step taken by a ray in an interior cell (at least k cells from both faces on every axis,
// k = the cells a full step may cross, at least 1; there the fraction is in [0, 1], as emission and
// every step path leave it) whose |T| components are at most tlim ends at least 4 kFaceMargin
// cells inside every face, so it is taken without the edge extension: its stage points stay
// inside the box (they leave the straight line by h^2 |D| / 2 in the step parameter, about 1e-7
// cells at the fields here).  That test is integer compares and one maximum.  A ray in a cell near
// the faces is tested on the straight end point of a full step: more than kFaceMargin inside, the
// full step is taken the same way; otherwise the exit rule decides, through the edge-extended
// sampling (a full step there, at fraction 1, gives the same bits as the inside one wherever both
// apply).  The exit-rule path leaves the state in a cell of the grid; a full step taken without the
// edge extension does so unless its path bends more than kFaceMargin cells off the straight line
// (a field far steeper than any here), and a state left outside the grid takes the exit rule next
// (both tests above check the cell index first), so the ray's own cell index is in the grid
// whenever it is used unclamped.
template <typename F, int NODES = 0>
__device__ __forceinline__ int trace_step(const TraceParams &P, CellCache &cc, int c[3], double fd[3], const F Tr[3],
                                          F dT[3], const StepGeom<F> &sg, int &steps)
{
    const F *g = sg.g;
    const int *last = sg.last;
    // bitwise, not short-circuit: one branch for the whole test.  A direction that is all NaN fails;
    // one with a NaN next to finite components may pass (fmax returns the number), and its step then
    // stays in bounds through the clamped cell indices.
    const F Tm = fmax(fmax(fabs(Tr[0] + dT[0]), fabs(Tr[1] + dT[1])), fabs(Tr[2] + dT[2]));
    const bool inside = ((unsigned)(c[0] - sg.lo[0]) < sg.bnd[0]) & ((unsigned)(c[1] - sg.lo[1]) < sg.bnd[1]) &
                        ((unsigned)(c[2] - sg.lo[2]) < sg.bnd[2]) & (Tm <= sg.tlim);
    if (__builtin_expect(inside, 1)) {
        rkn_step<F, true, true, NODES>(P, cc, c, fd, Tr, dT, sg, (F)1);
        return ++steps > P.max_steps ? STEP_LIMIT : STEP_GO;
    }
    // near the faces: the straight end point of a full step (a NaN counts as outside), from a
    // state whose cell is a cell of the grid.  (A step whose path bends more than kFaceMargin
    // cells off its straight line can end a hair outside the box with the index one past a face;
    // such a state takes the exit rule, whose sampling clamps every index.)
    bool far = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const F e = ((F)c[a] + (F)fd[a]) + g[a] * (Tr[a] + dT[a]);
        far = far & (e > (F)kFaceMargin) & (e < (F)last[a] - (F)kFaceMargin) & ((unsigned)c[a] < (unsigned)last[a]);
    }
    if (far) {
        rkn_step<F, true, true, NODES>(P, cc, c, fd, Tr, dT, sg, (F)1);
        return ++steps > P.max_steps ? STEP_LIMIT : STEP_GO;
    }
    F lam = (F)3.0e38;
    int ax = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const F v = g[a] * (Tr[a] + dT[a]);
        F l = (F)3.0e38;
        if (v > (F)0) l = (F)((double)(last[a] - c[a]) - fd[a]) / v;
        else if (v < (F)0) l = (F)((double)(-c[a]) - fd[a]) / v;
        if (l < lam) { lam = l; ax = a; }
    }
    const bool hit = ax >= 0 && lam <= (F)1;
    const bool up = hit && (pick3<F>(Tr, ax) + pick3<F>(dT, ax)) > (F)0;
    // one call site for both the partial step and the edge-extended full step
    if (!hit || lam > (F)0) {
        rkn_step<F, false, false, NODES>(P, cc, c, fd, Tr, dT, sg, hit ? lam : (F)1);
        ++steps;
        // a step ending on or a hair beyond the upper face leaves cell n - 1 at fraction ~0: keep the
        // index a cell of the grid (same position), as the inside steps assume
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int i = min(max(c[a], 0), last[a] - 1);
            fd[a] += (double)(c[a] - i);
            c[a] = i;
        }
    }
    if (!hit) return steps > P.max_steps ? STEP_LIMIT : STEP_GO;
    const F Tn[3] = {Tr[0] + dT[0], Tr[1] + dT[1], Tr[2] + dT[2]};
    const F Ta = pick3<F>(Tn, ax);
    if (up ? (Ta > (F)0) : (Ta < (F)0)) {
        const int la = pick3<int>(last, ax);
        const double target = up ? (double)la : 0.0;
        const double l2 = (target - ((double)pick3<int>(c, ax) + pick3<double>(fd, ax))) /
                          ((double)pick3<F>(g, ax) * (double)Ta);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (b == ax) {
                c[b] = up ? la - 1 : 0;
                fd[b] = up ? 1.0 : 0.0;
            } else {
                fd[b] += l2 * (double)g[b] * (double)Tn[b];
            }
        }
        return STEP_EXIT;
    }
    return steps > P.max_steps ? STEP_LIMIT : STEP_GO;  // turned back within the last step
}

// Integrate from the cell-local state until the ray leaves the box (see trace_step).  Returns the
// number of steps; sets *limited when max_steps is exceeded.
template <typename F, int NODES = 0>
__device__ __forceinline__ int trace_box(const TraceParams &P, CellCache &cc, int c[3], double fd[3],
                                         const F Tr[3], F dT[3], bool *limited)
{
    const StepGeom<F> sg = step_geom<F>(P);
    int steps = 0;
    for (;;) {
        const int r = trace_step<F, NODES>(P, cc, c, fd, Tr, dT, sg, steps);
        if (r != STEP_GO) {
            *limited = r == STEP_LIMIT;
            return steps;
        }
    }
}

// Ray-sphere intersection on the cap around the vertex.  Vertex at lens-frame z = zv, signed
// radius Rs (centre at zv + Rs).  H: hit point, N: unit normal facing -z near the axis.
__device__ __forceinline__ bool cap_hit(const double Pp[3], const double u[3], double zv,
                                        double Rs, double H[3], double N[3])
{
    #pragma clang fp contract(off)
    const double qx = Pp[0], qy = Pp[1], qz = Pp[2] - zv;
    const double b = qx * u[0] + qy * u[1] + qz * u[2] - Rs * u[2];
    const double cc = qx * qx + qy * qy + qz * qz - 2.0 * Rs * qz;
    const double disc = b * b - cc;
    if (!(disc >= 0.0)) return false;
    const double sq = sqrt(disc);
    const double den = b >= 0.0 ? -(b + sq) : -(b - sq);
    if (den == 0.0) return false;
    const double s = cc / den;  // the smaller root: the cap near the vertex
    H[0] = Pp[0] + s * u[0];
    H[1] = Pp[1] + s * u[1];
    H[2] = Pp[2] + s * u[2];
    const double ir = 1.0 / Rs;
    N[0] = H[0] * ir;
    N[1] = H[1] * ir;
    N[2] = (H[2] - zv - Rs) * ir;
    return true;
}

// Snell's law (eq. 7) in vector form; false on total internal reflection.
__device__ __forceinline__ bool snell(const double u[3], const double N[3], double n1, double n2,
                                      double out[3])
{
    #pragma clang fp contract(off)
    const double eta = n1 / n2;
    const double ci = -(u[0] * N[0] + u[1] * N[1] + u[2] * N[2]);
    const double k = 1.0 - eta * eta * (1.0 - ci * ci);
    if (k < 0.0) return false;
    const double m = eta * ci - sqrt(k);
    out[0] = eta * u[0] + m * N[0];
    out[1] = eta * u[1] + m * N[1];
    out[2] = eta * u[2] + m * N[2];
    return true;
}

// Aperture, both lens surfaces and the sensor plane (lens frame: z from the front vertex).
__device__ __forceinline__ int optics_to_sensor(const TraceParams &P, const double R[3], const double u[3],
                                double *xpx, double *ypx)
{
    #pragma clang fp contract(off)
    if (!(u[2] > 0.0)) return PBR_RAY_MISSED;
    const double s = (P.z_lens - R[2]) / u[2];
    double A[3] = {R[0] + s * u[0], R[1] + s * u[1], 0.0};
    if (A[0] * A[0] + A[1] * A[1] > P.a * P.a) return PBR_RAY_BLOCKED_APERTURE;
    double H1[3], N[3], v[3], w[3], H2[3];
    if (!cap_hit(A, u, 0.0, P.R, H1, N)) return PBR_RAY_BLOCKED_LENS;
    if (H1[0] * H1[0] + H1[1] * H1[1] > P.clear * P.clear) return PBR_RAY_BLOCKED_LENS;
    if (!snell(u, N, P.n_inf, P.n_glass, v)) return PBR_RAY_TIR;
    if (!cap_hit(H1, v, P.t, -P.R, H2, N)) return PBR_RAY_BLOCKED_LENS;
    if (H2[0] * H2[0] + H2[1] * H2[1] > P.clear * P.clear) return PBR_RAY_BLOCKED_LENS;
    if (!snell(v, N, P.n_glass, P.n_inf, w)) return PBR_RAY_TIR;
    if (!(w[2] > 0.0)) return PBR_RAY_MISSED;
    const double s2 = (P.z_sensor - P.z_lens - H2[2]) / w[2];
    *xpx = (H2[0] + s2 * w[0]) / P.pitch + 0.5 * (double)P.W;
    *ypx = (H2[1] + s2 * w[1]) / P.pitch + 0.5 * (double)P.H;
    return PBR_RAY_DEPOSITED;
}

__device__ __forceinline__ void atomic_add_u64(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ general optical chain (sec. 3.3)

// First intersection at s > 1e-12 along P + s u with the sphere of signed radius Rs whose vertex
// is (cx, cy, zv), on the half of the sphere facing its vertex; Rs = 0: the plane z = zv.  Writes
// the hit and the geometric normal (H - C) / Rs ((0, 0, -1) for a plane).
__device__ __forceinline__ bool chain_hit(const double P[3], const double u[3], double cx, double cy, double zv,
                                          double Rs, double H[3], double N[3])
{
    #pragma clang fp contract(off)
    const double eps = 1e-12;
    if (Rs == 0.0) {
        if (u[2] == 0.0) return false;
        const double s = (zv - P[2]) / u[2];
        if (!(s > eps)) return false;
        H[0] = P[0] + s * u[0];
        H[1] = P[1] + s * u[1];
        H[2] = zv;
        N[0] = 0.0; N[1] = 0.0; N[2] = -1.0;
        return true;
    }
    const double C[3] = {cx, cy, zv + Rs};
    const double d[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
    const double b = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    const double c = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - Rs * Rs;
    const double disc = b * b - c;
    if (disc < 0.0) return false;
    const double sq = sqrt(disc);
    const double q = -(b + (b >= 0.0 ? sq : -sq));  // roots q and c / q without cancellation
    const double ra = q, rb = q != 0.0 ? c / q : q;
    const double r1 = fmin(ra, rb), r2 = fmax(ra, rb);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double s = k ? r2 : r1;
        if (!(s > eps)) continue;
        const double h[3] = {P[0] + s * u[0], P[1] + s * u[1], P[2] + s * u[2]};
        if ((h[2] - C[2]) * Rs > 0.0) continue;  // the far half of the sphere
#pragma unroll
        for (int a = 0; a < 3; ++a) { H[a] = h[a]; N[a] = (h[a] - C[a]) / Rs; }
        return true;
    }
    return false;
}

// The ray from R along unit u through the chain's surfaces in order, then onto the sensor plane
// (refraction by eq. 7 with total internal reflection, reflection about the local normal, stops
// and rims blocking; a lenslet array refracts at the cap of the lenslet whose cell the ray meets).
__device__ int chain_to_sensor(const TraceParams &P, const double R[3], const double u0[3], double *xpx,
                               double *ypx)
{
    #pragma clang fp contract(off)
    const pbr_optical_chain &ch = *P.chain;
    double X[3] = {R[0], R[1], R[2]}, u[3] = {u0[0], u0[1], u0[2]};
    double n_cur = P.n_inf;
    for (int k = 0; k < ch.n_surfaces; ++k) {
        const pbr_surface f = ch.s[k];
        const bool stop = f.type == PBR_SURF_APERTURE;
        const int blocked = stop ? PBR_RAY_BLOCKED_APERTURE : PBR_RAY_BLOCKED_LENS;
        double cx = 0.0, cy = 0.0, H[3], N[3];
        if (f.type == PBR_SURF_LENSLETS) {  // the lenslet whose square cell the ray enters
            if (!chain_hit(X, u, 0.0, 0.0, f.z, 0.0, H, N)) return PBR_RAY_BLOCKED_LENS;
            cx = f.pitch * floor(H[0] / f.pitch + 0.5);
            cy = f.pitch * floor(H[1] / f.pitch + 0.5);
        }
        if (!chain_hit(X, u, cx, cy, f.z, stop ? 0.0 : f.radius, H, N)) return blocked;
        if (H[0] * H[0] + H[1] * H[1] > f.clear * f.clear) return blocked;
        if (f.type == PBR_SURF_LENSLETS && (fabs(H[0] - cx) > 0.5 * f.pitch || fabs(H[1] - cy) > 0.5 * f.pitch))
            return PBR_RAY_BLOCKED_LENS;
        if (u[0] * N[0] + u[1] * N[1] + u[2] * N[2] > 0.0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
        if (f.type == PBR_SURF_MIRROR) {
            const double dn = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) u[a] = u[a] - 2.0 * dn * N[a];
        } else if (!stop) {
            const double n_next = f.n_after > 0.0 ? f.n_after : P.n_inf;
            double v[3];
            if (!snell(u, N, n_cur, n_next, v)) return PBR_RAY_TIR;
            const double vl = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) u[a] = v[a] / vl;
            n_cur = n_next;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) X[a] = H[a];
    }
    if (u[2] == 0.0) return PBR_RAY_MISSED;
    const double s = (P.z_sensor - X[2]) / u[2];
    if (!(s > 0.0)) return PBR_RAY_MISSED;
    *xpx = (X[0] + s * u[0]) / P.pitch + 0.5 * (double)P.W;
    *ypx = (X[1] + s * u[1]) / P.pitch + 0.5 * (double)P.H;
    return PBR_RAY_DEPOSITED;
}

// ------------------------------------------------------------------ kernel 1: emission, entry

// sec. 3.1: ray j of source s aims at the aperture point (a sqrt(u1) cos 2 pi u2,
// a sqrt(u1) sin 2 pi u2) of the front-vertex plane; (u1, u2) are the two 24-bit fields of
// SplitMix64 output number (s << 32 | j).  The ray goes straight to the box (slab test) and its
// state is written cell-local; a ray that never enters keeps its world position and direction.
// Source position S and unit direction u of ray rid as it leaves its source.
__device__ __forceinline__ void initial_direction(const TraceParams &P, int64_t rid, double S[3], double u[3])
{
    #pragma clang fp contract(off)
    int64_t s = rid / P.rays_per_src;
    const int32_t j = (int32_t)(rid - s * P.rays_per_src);
    if (PBR_CHECKED && !access_ok(P, s >= 0 && s < P.n_src)) s = s < 0 ? 0 : P.n_src - 1;
    const float4 sv = P.src[s];
    S[0] = (double)sv.x;
    S[1] = (double)sv.y;
    S[2] = (double)sv.z;
    const uint64_t hsh = splitmix64_at(P.seed, ((uint64_t)s << 32) | (uint64_t)(uint32_t)j);
    const double u1 = (double)(hsh >> 40) * (1.0 / 16777216.0);
    const double u2 = (double)((hsh >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0);
    const double rr = P.a * sqrt(u1);
    double sn, cs;
    sincos(kTwoPi * u2, &sn, &cs);
    u[0] = rr * cs - S[0];
    u[1] = rr * sn - S[1];
    u[2] = P.z_lens - S[2];
    const double il = 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    u[0] *= il; u[1] *= il; u[2] *= il;
}

// Mie factor of a ray leaving its source along u (sec. 3.1): the intensity table at the
// scattering angle acos(u . laser), linear between its nodes theta_k = k pi / (mie_n - 1).
__device__ __forceinline__ double mie_weight(const TraceParams &P, const double u[3])
{
    #pragma clang fp contract(off)
    double c = u[0] * P.laser[0] + u[1] * P.laser[1] + u[2] * P.laser[2];
    c = fmin(fmax(c, -1.0), 1.0);
    const double t = acos(c) / 3.14159265358979323846 * (double)(P.mie_n - 1);
    int i = min((int)floor(t), P.mie_n - 2);
    if (PBR_CHECKED && !access_ok(P, i >= 0)) i = 0;
    const double f = t - (double)i;
    return P.mie[i] * (1.0 - f) + P.mie[i + 1] * f;
}

// Key of the ray at position q of the processing order.  With a source order, position q is ray
// q mod rays_per_src of source order[q / rays_per_src] (clamped into range), and the key is that
// ray's position without the order: everything the ray is (random numbers, weight, record index,
// per-source sums) follows from the key, so the order changes nothing but the schedule.
__device__ __forceinline__ int64_t ray_key(const TraceParams &P, int64_t q)
{
    if (!P.order) return q;
    const int64_t k = q / P.rays_per_src;
    if (PBR_CHECKED && !access_ok(P, k >= 0 && k < P.n_src)) return q;
    int64_t s = P.order[k];
    if (PBR_CHECKED) access_ok(P, s >= 0 && s < P.n_src);  // an entry that is no source index is counted
    s = s < 0 ? 0 : (s >= P.n_src ? P.n_src - 1 : s);
    return s * P.rays_per_src + (q - k * P.rays_per_src);
}

__device__ __forceinline__ void emit_ray(const TraceParams &P, int64_t rid, RayState &r)
{
    // FP64 set-up and optics: no contracted multiply-adds, so every kernel that inlines this
    // (single-image and batched paths) computes the same bits
    #pragma clang fp contract(off)
    double S[3], u[3];
    initial_direction(P, rid, S, u);
    double Rw[3] = {S[0], S[1], S[2]};
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && S[a] >= P.lo[a] && S[a] <= P.hi[a];
    bool entered = inside;
    int eax = -1;
    if (!inside) {
        double tn = -1.0e308, tf = 1.0e308;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (u[a] != 0.0) {
                const double t1 = (P.lo[a] - S[a]) / u[a], t2 = (P.hi[a] - S[a]) / u[a];
                const double nr = t1 < t2 ? t1 : t2, fr = t1 < t2 ? t2 : t1;
                if (nr > tn) { tn = nr; eax = a; }
                if (fr < tf) tf = fr;
            } else if (S[a] < P.lo[a] || S[a] > P.hi[a]) {
                ok = false;
            }
        }
        if (ok && eax >= 0 && tn <= tf && tn >= 0.0) {
            entered = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) Rw[a] = S[a] + tn * u[a];
        }
    }
    if (!entered) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.fd[a] = Rw[a];
            r.Tr[a] = (float)u[a];
            r.dT[a] = (float)(u[a] - (double)r.Tr[a]);  // direction kept as a float hi/lo pair
            r.c[a] = 0;
        }
        r.info = 0;
        return;
    }
    const int nn[3] = {P.nx, P.ny, P.nz};
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = (Rw[a] - P.origin[a]) / P.spacing[a];
        if (a == eax) p = u[a] > 0.0 ? 0.0 : (double)(nn[a] - 1);
        p = p < 0.0 ? 0.0 : p;
        p = p > (double)(nn[a] - 1) ? (double)(nn[a] - 1) : p;
        int ci = (int)floor(p);
        ci = ci > nn[a] - 2 ? nn[a] - 2 : ci;
        r.c[a] = ci;
        r.fd[a] = p - (double)ci;
        f[a] = (float)r.fd[a];
    }
    // inside: T = n dR/ds = n u (eq. 4), n interpolated at the entry point
    CellCache cc;
    cc.ix = -1;
    float G0[3];
    const float n0 = P.node_layout ? sample_field<float, false, false, true>(P, cc, r.c, f, G0)
                                   : sample_field<float>(P, cc, r.c, f, G0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {  // T0 as a float hi/lo pair: no rounding of the entry direction
        const double T0 = (double)n0 * u[a];
        r.Tr[a] = (float)T0;
        r.dT[a] = (float)(T0 - (double)r.Tr[a]);
    }
    r.info = RS_ENTERED;
}

__global__ void __launch_bounds__(256) k_emit(TraceParams P, RayState *__restrict__ st, int64_t first,
                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    RayState r;
    emit_ray(P, ray_key(P, first + i), r);
    st[i] = r;
}

// ------------------------------------------------------------------ kernel 2: the ray equation

template <typename F, int NODES = 0>
__device__ __forceinline__ void box_ray(const TraceParams &P, RayState &r)
{
    // T = Tr + dT; in FP32 the low part of the entry direction starts the accumulated change
    F Tr[3], dT[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (sizeof(F) == sizeof(float)) {
            Tr[a] = (F)r.Tr[a];
            dT[a] = (F)r.dT[a];
        } else {
            Tr[a] = (F)((double)r.Tr[a] + (double)r.dT[a]);
            dT[a] = (F)0;
        }
    }
    CellCache cc;
    cc.ix = -1;
    bool limited = false;
    const int steps = trace_box<F, NODES>(P, cc, r.c, r.fd, Tr, dT, &limited);
    // exit direction as a float hi/lo pair (about 48 significant bits)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double T = (double)Tr[a] + (double)dT[a];
        r.Tr[a] = (float)T;
        r.dT[a] = (float)(T - (double)r.Tr[a]);
    }
    r.info = RS_ENTERED | (limited ? RS_LIMITED : 0) | (steps << RS_STEP_SHIFT);
}

// Ray i = k, or i = list[k] for k < *count when a list is given (the rays the surrogate left to
// the tracer, packed densely so that waves are not held by a few scattered rays).
__device__ __forceinline__ bool box_index(int64_t n, const int *__restrict__ list,
                                          const unsigned long long *__restrict__ count, int64_t *i)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (list) {
        const unsigned long long m = *count;
        if ((unsigned long long)k >= m) return false;
        *i = list[k];
        return true;
    }
    *i = k;
    return k < n;
}

template <typename F, int NODES = 0>
__device__ __forceinline__ void box_body(const TraceParams &P, RayState *__restrict__ st, int64_t n,
                                         const int *__restrict__ list, const unsigned long long *__restrict__ count)
{
    int64_t i;
    if (!box_index(n, list, count, &i)) return;
    RayState r = st[i];
    if ((r.info & (RS_ENTERED | RS_SURR)) != RS_ENTERED) return;
    box_ray<F, NODES>(P, r);
    st[i] = r;
}

// FP32 integration: 88 VGPRs, five waves per SIMD.  NODES: field stored per node (the corner gather
// needs more registers: four waves per SIMD).
template <bool NODES = false>
__global__ void __launch_bounds__(256, NODES ? 4 : 5) k_box32(TraceParams P, RayState *__restrict__ st, int64_t n,
                                                  const int *__restrict__ list,
                                                  const unsigned long long *__restrict__ count)
{
    box_body<float, NODES>(P, st, n, list, count);
}

template <bool NODES = false>
__global__ void __launch_bounds__(256) k_box64(TraceParams P, RayState *__restrict__ st, int64_t n,
                                               const int *__restrict__ list,
                                               const unsigned long long *__restrict__ count)
{
    box_body<double, NODES>(P, st, n, list, count);
}

// Persistent FP32 integration with lane refill: a fixed grid of waves (five per SIMD) takes rays
// from one queue; a lane whose ray has left the box takes the next one at once, one atomic per
// wave for all lanes that need a ray, so that short and long paths do not leave lanes idle until
// the longest ray of a wave is done.  Same per-ray arithmetic as k_box32 (bit-identical states).
// *queue must be zero at launch; every wave leaves once the queue is drained and its lanes idle.
__global__ void __launch_bounds__(256, 5) k_box32_refill(TraceParams P, RayState *__restrict__ st, int64_t n,
                                                         const int *__restrict__ list,
                                                         const unsigned long long *__restrict__ count,
                                                         unsigned long long *__restrict__ queue)
{
    if (P.node_layout) return;  // cell records only (the host never launches it otherwise)
    const int lane = threadIdx.x & 63;
    const unsigned long long total = list ? *count : (unsigned long long)n;
    const StepGeom<float> sg = step_geom<float>(P);
    int64_t i = -1;  // this lane's ray, -1: none
    RayState r;
    float Tr[3], dT[3];
    CellCache cc;
    int steps = 0;
    bool drained = false;  // the queue had nothing left for this wave
    for (;;) {
        const bool need = i < 0;
        const unsigned long long want = __ballot(need);
        if (want && !drained) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(queue, (unsigned long long)__popcll(want));
            base = __shfl(base, 0);
            if (base + (unsigned long long)__popcll(want) >= total) drained = true;
            if (need) {
                const unsigned long long k = base + __popcll(want & ((1ull << lane) - 1ull));
                if (k < total) {
                    const int64_t j = list ? (int64_t)list[k] : (int64_t)k;
                    r = st[j];
                    if ((r.info & (RS_ENTERED | RS_SURR)) == RS_ENTERED) {
                        i = j;
#pragma unroll
                        for (int a = 0; a < 3; ++a) { Tr[a] = r.Tr[a]; dT[a] = r.dT[a]; }
                        cc.ix = -1;
                        steps = 0;
                    }
                }
            }
            continue;  // lanes that drew a ray with nothing to integrate draw again
        }
        if (__ballot(i >= 0) == 0) break;  // queue drained and no lane busy
        if (i >= 0) {
            const int res = trace_step<float>(P, cc, r.c, r.fd, Tr, dT, sg, steps);
            if (res != STEP_GO) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double T = (double)Tr[a] + (double)dT[a];
                    r.Tr[a] = (float)T;
                    r.dT[a] = (float)(T - (double)r.Tr[a]);
                }
                r.info = RS_ENTERED | (res == STEP_LIMIT ? RS_LIMITED : 0) | (steps << RS_STEP_SHIFT);
                st[i] = r;
                i = -1;
            }
        }
    }
}

// ------------------------------------------------------------------ mixed precision

// FP64 flag of the brick holding cell c (cell clamped onto the grid).
__device__ __forceinline__ bool brick_is_fp64(const TraceParams &P, const int c[3])
{
    const int bx = min(max(c[0], 0), P.nx - 2) / kBrick;
    const int by = min(max(c[1], 0), P.ny - 2) / kBrick;
    const int bz = min(max(c[2], 0), P.nz - 2) / kBrick;
    if (PBR_CHECKED && !access_ok(P, bx < P.nbx && by < P.nby && bz < P.nbz)) return true;
    return P.brick_fp64[((size_t)bz * P.nby + by) * P.nbx + bx] != 0;
}

// One step in FP64 from the FP32 state: T = Tr + dT is carried in double through the step, then
// split again into a float hi/lo pair.
template <bool FULL, int NODES>
__device__ __forceinline__ void rkn_step_fp64(const TraceParams &P, CellCache &cc, int c[3], double fd[3],
                                              float Tr[3], float dT[3], double lam)
{
    double T64[3], d64[3] = {0.0, 0.0, 0.0};
    const StepGeom<double> sg64 = step_geom<double>(P);
#pragma unroll
    for (int a = 0; a < 3; ++a) T64[a] = (double)Tr[a] + (double)dT[a];
    rkn_step<double, FULL, false, NODES>(P, cc, c, fd, T64, d64, sg64, lam);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double T = T64[a] + d64[a];
        Tr[a] = (float)T;
        dT[a] = (float)(T - (double)Tr[a]);
    }
}

// trace_box<float> with the step precision chosen per step from the brick of the current cell.
template <int NODES>
__device__ __forceinline__ int trace_box_mixed(const TraceParams &P, CellCache &cc, int c[3], double fd[3],
                                               float Tr[3], float dT[3], bool *limited, int *n64)
{
    const StepGeom<float> sg = step_geom<float>(P);
    const float *g = sg.g;
    const int *last = sg.last;
    int steps = 0;
    *limited = false;
    for (;;) {
        bool near = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = g[a] * (Tr[a] + dT[a]);
            const float fa = (float)fd[a];
            near = near || (v > 0.0f && (float)(last[a] - c[a]) - fa <= v) || (v < 0.0f && (float)(-c[a]) - fa >= v);
        }
        if (near) {
            float lam = 3.0e38f;
            int ax = -1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float v = g[a] * (Tr[a] + dT[a]);
                float l = 3.0e38f;
                if (v > 0.0f) l = (float)((double)(last[a] - c[a]) - fd[a]) / v;
                else if (v < 0.0f) l = (float)((double)(-c[a]) - fd[a]) / v;
                if (l < lam) { lam = l; ax = a; }
            }
            if (ax >= 0 && lam <= 1.0f) {
                const bool up = (pick3<float>(Tr, ax) + pick3<float>(dT, ax)) > 0.0f;
                if (lam > 0.0f) {
                    if (brick_is_fp64(P, c)) { rkn_step_fp64<false, NODES>(P, cc, c, fd, Tr, dT, (double)lam); ++*n64; }
                    else rkn_step<float, false, false, NODES>(P, cc, c, fd, Tr, dT, sg, lam);
                    ++steps;
                }
                const float Tn[3] = {Tr[0] + dT[0], Tr[1] + dT[1], Tr[2] + dT[2]};
                const float Ta = pick3<float>(Tn, ax);
                if (up ? (Ta > 0.0f) : (Ta < 0.0f)) {
                    const int la = pick3<int>(last, ax);
                    const double target = up ? (double)la : 0.0;
                    const double l2 = (target - ((double)pick3<int>(c, ax) + pick3<double>(fd, ax))) /
                                      ((double)pick3<float>(g, ax) * (double)Ta);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        if (b == ax) {
                            c[b] = up ? la - 1 : 0;
                            fd[b] = up ? 1.0 : 0.0;
                        } else {
                            fd[b] += l2 * (double)g[b] * (double)Tn[b];
                        }
                    }
                    return steps;
                }
                if (steps > P.max_steps) { *limited = true; return steps; }
                continue;
            }
        }
        if (brick_is_fp64(P, c)) { rkn_step_fp64<true, NODES>(P, cc, c, fd, Tr, dT, 1.0); ++*n64; }
        else rkn_step<float, true, false, NODES>(P, cc, c, fd, Tr, dT, sg, 1.0f);
        if (++steps > P.max_steps) { *limited = true; return steps; }
    }
}

template <bool NODES>
__global__ void __launch_bounds__(256) k_box_mixed(TraceParams P, RayState *__restrict__ st, int64_t n,
                                                   const int *__restrict__ list,
                                                   const unsigned long long *__restrict__ count)
{
    __shared__ unsigned long long s64;
    if (threadIdx.x == 0) s64 = 0ull;
    __syncthreads();
    int64_t i;
    const bool live = box_index(n, list, count, &i);
    int n64 = 0;
    if (live) {
        RayState r = st[i];
        if ((r.info & (RS_ENTERED | RS_SURR)) == RS_ENTERED) {
            float Tr[3] = {r.Tr[0], r.Tr[1], r.Tr[2]}, dT[3] = {r.dT[0], r.dT[1], r.dT[2]};
            CellCache cc;
            cc.ix = -1;
            bool limited = false;
            const int steps = trace_box_mixed<NODES ? 2 : 0>(P, cc, r.c, r.fd, Tr, dT, &limited, &n64);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double T = (double)Tr[a] + (double)dT[a];
                r.Tr[a] = (float)T;
                r.dT[a] = (float)(T - (double)r.Tr[a]);
            }
            r.info = RS_ENTERED | (limited ? RS_LIMITED : 0) | (steps << RS_STEP_SHIFT);
            st[i] = r;
        }
    }
    if (n64) atomicAdd(&s64, (unsigned long long)n64);
    __syncthreads();
    if (threadIdx.x == 0 && s64) atomic_add_u64(P.counters + CNT_STEPS64, s64);
}

// Calibration of the precision policy: each block samples one brick.  Sample ray k starts at a
// uniform point of the brick, aimed at a uniform point of the aperture, and is integrated over
// n_steps full steps in FP32 and in FP64 from the same state.  The two results are compared where
// they matter on the sensor: the apparent source point on the focused plane, times |M| / pitch.
template <bool NODES>
__global__ void __launch_bounds__(256) k_calibrate(TraceParams P, const int *__restrict__ bricks,
                                                   int n_steps, uint64_t seed, double z_focus,
                                                   double px_per_m, float *__restrict__ err)
{
    __shared__ unsigned s_err;
    if (threadIdx.x == 0) s_err = 0u;
    __syncthreads();
    const int b = bricks[blockIdx.x];
    const int bb[3] = {b % P.nbx, (b / P.nbx) % P.nby, b / (P.nbx * P.nby)};
    const int nn[3] = {P.nx, P.ny, P.nz};
    const uint64_t h1 = splitmix64_at(seed, ((uint64_t)(uint32_t)b << 32) | (2u * threadIdx.x));
    const uint64_t h2 = splitmix64_at(seed, ((uint64_t)(uint32_t)b << 32) | (2u * threadIdx.x + 1u));
    const double uu[5] = {(double)(h1 >> 40) * (1.0 / 16777216.0), (double)((h1 >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0),
                          (double)(h2 >> 40) * (1.0 / 16777216.0), (double)((h2 >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0),
                          (double)(h1 & 0xFFFFull) * (1.0 / 65536.0)};
    int c[3];
    double fd[3], X[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = (double)(bb[a] * kBrick) + (double)kBrick * uu[a];
        p = p > (double)(nn[a] - 1) ? (double)(nn[a] - 1) : p;
        int ci = (int)floor(p);
        ci = ci > nn[a] - 2 ? nn[a] - 2 : ci;
        c[a] = ci;
        fd[a] = p - (double)ci;
        f[a] = (float)fd[a];
        X[a] = P.origin[a] + p * P.spacing[a];
    }
    const double rr = P.a * sqrt(uu[3]);
    double sn, cs;
    sincos(kTwoPi * uu[4], &sn, &cs);
    double u[3] = {rr * cs - X[0], rr * sn - X[1], P.z_lens - X[2]};
    const double il = 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] *= il;
    CellCache cc;
    cc.ix = -1;
    float G0[3];
    const float n0 = sample_field<float, false, false, NODES ? 2 : 0>(P, cc, c, f, G0);
    // FP32
    int c32[3] = {c[0], c[1], c[2]};
    double fd32[3] = {fd[0], fd[1], fd[2]};
    float Tr[3], dT[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double T0 = (double)n0 * u[a];
        Tr[a] = (float)T0;
        dT[a] = (float)(T0 - (double)Tr[a]);
    }
    const StepGeom<float> sg = step_geom<float>(P);
    for (int k = 0; k < n_steps; ++k) rkn_step<float, true, false, NODES ? 2 : 0>(P, cc, c32, fd32, Tr, dT, sg, 1.0f);
    // FP64
    int c64[3] = {c[0], c[1], c[2]};
    double fd64[3] = {fd[0], fd[1], fd[2]};
    double T64[3], d64[3] = {0.0, 0.0, 0.0};
    const StepGeom<double> sg64 = step_geom<double>(P);
#pragma unroll
    for (int a = 0; a < 3; ++a) T64[a] = (double)n0 * u[a];
    cc.ix = -1;
    for (int k = 0; k < n_steps; ++k) rkn_step<double, true, false, NODES ? 2 : 0>(P, cc, c64, fd64, T64, d64, sg64, 1.0);
    double q32[2], q64[2];
    {
        double Xa[3], Xb[3], da[3], db[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Xa[a] = P.origin[a] + ((double)c32[a] + fd32[a]) * P.spacing[a];
            Xb[a] = P.origin[a] + ((double)c64[a] + fd64[a]) * P.spacing[a];
            da[a] = (double)Tr[a] + (double)dT[a];
            db[a] = T64[a] + d64[a];
        }
        const double ta = (Xa[2] - z_focus) / da[2], tb = (Xb[2] - z_focus) / db[2];
        q32[0] = Xa[0] - ta * da[0]; q32[1] = Xa[1] - ta * da[1];
        q64[0] = Xb[0] - tb * db[0]; q64[1] = Xb[1] - tb * db[1];
    }
    const double e = px_per_m * sqrt((q32[0] - q64[0]) * (q32[0] - q64[0]) + (q32[1] - q64[1]) * (q32[1] - q64[1]));
    const float ef = (float)e;
    if (ef > 0.0f) atomicMax(&s_err, __float_as_uint(ef));
    __syncthreads();
    if (threadIdx.x == 0) err[blockIdx.x] = __uint_as_float(s_err);
}

// ------------------------------------------------------------------ kernel 3: lens, sensor, spot

// Spot of one ray (sec. 3.4): fractions of a Gaussian of sigma_px centred at (x, y) over the
// pixels of the (2R+1)^2 window around the hit pixel, each the product of two erf differences,
// times the source weight, rounded to Q32.32.  Pixels inside the block's LDS tile are summed
// there first (integer adds, so the order does not matter); the others go straight to HBM.
template <int RF, int TILE>
__device__ __forceinline__ void deposit(const TraceParams &P, double x, double y, double w,
                                        unsigned long long *tile, int tx0, int ty0)
{
    #pragma clang fp contract(off)
    const int i0 = (int)x, j0 = (int)y;
    const double inv = 1.0 / (1.4142135623730950488 * P.sigma_px);
    float ex[2 * RF + 2], ey[2 * RF + 2];
#pragma unroll
    for (int m = 0; m < 2 * RF + 2; ++m) {
        ex[m] = erff((float)(((double)(i0 - RF + m) - x) * inv));
        ey[m] = erff((float)(((double)(j0 - RF + m) - y) * inv));
    }
    const float wf = (float)w;
#pragma unroll
    for (int dj = 0; dj <= 2 * RF; ++dj) {
        const int jj = j0 - RF + dj;
        if (jj < 0 || jj >= P.H) continue;
        const float fy = 0.5f * (ey[dj + 1] - ey[dj]) * wf;
#pragma unroll
        for (int di = 0; di <= 2 * RF; ++di) {
            const int ii = i0 - RF + di;
            if (ii < 0 || ii >= P.W) continue;
            const float cval = 0.5f * (ex[di + 1] - ex[di]) * fy;
            if (!(cval > 0.0f)) continue;
            const unsigned long long q = (unsigned long long)rint((double)cval * kTwoPow32);
            if (!q) continue;
            const int lx = ii - tx0, ly = jj - ty0;
            if ((unsigned)lx < (unsigned)TILE && (unsigned)ly < (unsigned)TILE)
                atomicAdd(tile + ly * TILE + lx, q);
            else
                atomic_add_u64(P.accum + (size_t)jj * (size_t)P.W + ii, q);
        }
    }
}

// Adds the sensor hits of this wave's deposited rays (on) into the per-source sums.  The rays of
// a source are consecutive, so the wave holds a few runs of one source index each: every run is
// summed across the wave and added by its first lane.  Integer sums (hits in units of 2^-24
// pixel): the result does not depend on the order in which rays arrive.  Wave-uniform control.
__device__ __forceinline__ void add_source_sums(const TraceParams &P, bool on, int64_t rid, double xpx,
                                                double ypx)
{
    const int64_t s = rid / P.rays_per_src;
    const long long qx = on ? (long long)rint(xpx * 16777216.0) : 0ll;
    const long long qy = on ? (long long)rint(ypx * 16777216.0) : 0ll;
    unsigned long long pending = __ballot(on);
    while (pending) {
        const int lead = __ffsll((unsigned long long)pending) - 1;
        const int64_t s0 = __shfl(s, lead, 64);
        const bool mine = on && s == s0;
        long long vx = mine ? qx : 0ll, vy = mine ? qy : 0ll, c = mine ? 1ll : 0ll;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            vx += __shfl_xor(vx, o, 64);
            vy += __shfl_xor(vy, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if ((int)__lane_id() == lead && (!PBR_CHECKED || access_ok(P, s0 >= 0 && s0 < P.n_src))) {
            pbr_source_sum *d = P.src_sums + s0;
            atomic_add_u64((unsigned long long *)&d->sum_x, (unsigned long long)vx);
            atomic_add_u64((unsigned long long *)&d->sum_y, (unsigned long long)vy);
            atomic_add_u64((unsigned long long *)&d->hits, (unsigned long long)c);
        }
        pending &= ~__ballot(mine);
    }
}

// Shared memory of the finish step of one block.
template <int TILE>
struct FinishShared {
    unsigned long long tile[TILE * TILE];
    unsigned long long cnt[CNT_SLOTS];
    int lead, tx0, ty0;
};

// Lens, sensor, spot, records and counters for the rays [first + base, first + base + 256) of one
// image, whose states are st[base ..]; rays at or beyond n are padding.  All threads of the block
// take part (barriers inside).
// RFX: footprint radius fixed at compile time (1..8), or 0 to switch on P.rfp per call (batches,
// whose images differ).  A fixed radius keeps the spot arrays, and so the register count, small.
// FEAT: optional steps compiled in only where used (each costs registers): bit 0 the Mie weighting,
// bit 1 a general optical chain in place of the singlet.
enum : int { FEAT_MIE = 1, FEAT_CHAIN = 2 };
template <int TILE, int RFX = 0, int FEAT = 0>
__device__ __forceinline__ void finish_block(const TraceParams &P, const RayState *__restrict__ st,
                                             int64_t first, int64_t base, int64_t n, FinishShared<TILE> &sh)
{
    #pragma clang fp contract(off)
    for (int q = threadIdx.x; q < TILE * TILE; q += blockDim.x) sh.tile[q] = 0ull;
    if (threadIdx.x == 0) sh.lead = 0x7fffffff;
    __syncthreads();

    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    int status = PBR_RAY_MISSED, nsteps = 0;
    bool entered = false;
    double Rw[3] = {0, 0, 0}, dir[3] = {0, 0, 1}, xpx = 0.0, ypx = 0.0;
    if (valid) {
        const RayState r = st[i];
        entered = (r.info & RS_ENTERED) != 0;
        nsteps = entered ? (r.info >> RS_STEP_SHIFT) : 0;
        status = PBR_RAY_DEPOSITED;
        double tn2 = 0.0, T[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Rw[a] = entered ? P.origin[a] + ((double)r.c[a] + r.fd[a]) * P.spacing[a] : r.fd[a];
            T[a] = (double)r.Tr[a] + (double)r.dT[a];
            tn2 += T[a] * T[a];
        }
        const double it = 1.0 / sqrt(tn2);
#pragma unroll
        for (int a = 0; a < 3; ++a) dir[a] = T[a] * it;
        if (r.info & RS_LIMITED) status = PBR_RAY_STEP_LIMIT;
        if (status == PBR_RAY_DEPOSITED)
            status = ((FEAT & FEAT_CHAIN) && P.chain) ? chain_to_sensor(P, Rw, dir, &xpx, &ypx)
                                                      : optics_to_sensor(P, Rw, dir, &xpx, &ypx);
        if (status == PBR_RAY_DEPOSITED &&
            !(xpx >= 0.0 && ypx >= 0.0 && xpx < (double)P.W && ypx < (double)P.H))
            status = PBR_RAY_OFF_SENSOR;
        if (status == PBR_RAY_DEPOSITED) atomicMin(&sh.lead, (int)threadIdx.x);
    }
    __syncthreads();
    // the block's first deposited ray anchors the tile: rays of one source land close together
    if ((int)threadIdx.x == sh.lead) {
        sh.tx0 = (int)xpx - TILE / 2;
        sh.ty0 = (int)ypx - TILE / 2;
    }
    __syncthreads();
    const int64_t rid = valid ? ray_key(P, first + i) : first + i;
    if (P.src_sums) add_source_sums(P, valid && status == PBR_RAY_DEPOSITED, rid, xpx, ypx);
    if (valid && status == PBR_RAY_DEPOSITED) {
        int64_t s = rid / P.rays_per_src;
        if (PBR_CHECKED && !access_ok(P, s >= 0 && s < P.n_src)) s = s < 0 ? 0 : P.n_src - 1;
        const float4 sv = P.src[s];
        double w = sv.w > 0.0f ? (sv.w < 1.0f ? (double)sv.w : 1.0) : 0.0;  // weights in [0, 1]
        if ((FEAT & FEAT_MIE) && P.mie) {  // the ray's Mie factor, from its direction at the source
            double S0[3], u0[3];
            initial_direction(P, rid, S0, u0);
            w *= mie_weight(P, u0);
        }
        const int tx0 = sh.tx0, ty0 = sh.ty0;
        if (RFX > 0) deposit<(RFX > 0 ? RFX : 1), TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0);
        else switch (P.rfp) {
            case 1: deposit<1, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 2: deposit<2, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 3: deposit<3, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 4: deposit<4, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 5: deposit<5, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 6: deposit<6, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            case 7: deposit<7, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
            default: deposit<8, TILE>(P, xpx, ypx, w, sh.tile, tx0, ty0); break;
        }
    }
    if (valid) {
        if (P.record && rid >= P.rec_first) {
            const int64_t off = rid - P.rec_first;
            const int64_t k = off / P.rec_stride;
            if (k * P.rec_stride == off && k < P.rec_max) {
                pbr_ray_exit e;
                e.ray_id = rid;
                e.status = status;
                e.n_steps = nsteps;
                e.entered = entered ? 1 : 0;
                e.reserved = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) { e.vol_exit_pos[a] = Rw[a]; e.vol_exit_dir[a] = dir[a]; }
                e.sensor_px[0] = xpx;
                e.sensor_px[1] = ypx;
                P.rec[k] = e;
            }
        }
        atomicAdd(&sh.cnt[CNT_STATUS + status], 1ull);
        if (entered) atomicAdd(&sh.cnt[CNT_ENTERED], 1ull);
        atomicAdd(&sh.cnt[CNT_STEPS], (unsigned long long)nsteps);
    }
    __syncthreads();
    // flush the tile: one global atomic per touched pixel
    if (sh.lead != 0x7fffffff) {
        const int tx0 = sh.tx0, ty0 = sh.ty0;
        for (int q = threadIdx.x; q < TILE * TILE; q += blockDim.x) {
            const unsigned long long v = sh.tile[q];
            if (PBR_CHECKED && v &&
                !access_ok(P, (unsigned)(ty0 + q / TILE) < (unsigned)P.H && (unsigned)(tx0 + q % TILE) < (unsigned)P.W))
                continue;
            if (v) atomic_add_u64(P.accum + (size_t)(ty0 + q / TILE) * (size_t)P.W + (tx0 + q % TILE), v);
        }
    }
    __syncthreads();
}

template <int TILE>
__device__ __forceinline__ void flush_counters(const TraceParams &P, FinishShared<TILE> &sh)
{
    if (threadIdx.x < CNT_STEPS + 1 && sh.cnt[threadIdx.x] != 0ull)
        atomic_add_u64(P.counters + threadIdx.x, sh.cnt[threadIdx.x]);
}

template <int TILE, int RF, int FEAT = 0>
__global__ void __launch_bounds__(256) k_finish(TraceParams P, const RayState *__restrict__ st,
                                                int64_t first, int64_t n)
{
    __shared__ FinishShared<TILE> sh;
    if (threadIdx.x < CNT_SLOTS) sh.cnt[threadIdx.x] = 0ull;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x)
        finish_block<TILE, RF, FEAT>(P, st, first, base, n, sh);
    flush_counters<TILE>(P, sh);
}

// ------------------------------------------------------------------ batches of images

// Segment of one round of a batch: rays [first_ray, first_ray + n_rays) of image `image`, whose
// states start at slot slot_base (a slot = 256 rays; segments are padded to whole slots).
__device__ __forceinline__ int find_segment(const BatchSeg *__restrict__ segs, int nseg, int64_t slot)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // last segment with slot_base <= slot
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].slot_base <= slot) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_emit_batch(const TraceParams *__restrict__ params,
                                                    const BatchSeg *__restrict__ segs, int nseg,
                                                    RayState *__restrict__ st)
{
    const int k = __builtin_amdgcn_readfirstlane(find_segment(segs, nseg, blockIdx.x));
    const BatchSeg sg = segs[k];
    const int64_t local = (int64_t)(blockIdx.x - sg.slot_base) * 256 + threadIdx.x;
    if (local >= sg.n_rays) return;
    RayState r;
    emit_ray(params[sg.image], ray_key(params[sg.image], sg.first_ray + local), r);
    st[(int64_t)blockIdx.x * 256 + threadIdx.x] = r;
}

// Persistent integration over one round: every wave pulls the next unit of `unit_rays` rays
// (64, 128 or 256: units never straddle a slot) from a global counter until none is left.
// Segments are ordered by decreasing estimated cost, so long rays start first.  NODES: the
// images whose field is stored per node (their own counter, queue[1]; the per-cell images use
// queue[0]); each kernel passes over the other layout's units.
template <int BLOCK, bool NODES>
__global__ void __launch_bounds__(BLOCK, NODES ? 4 : 5) k_box_batch(const TraceParams *__restrict__ params,
                                                                    const BatchSeg *__restrict__ segs, int nseg,
                                                                    RayState *__restrict__ st, unsigned *queue,
                                                                    unsigned n_units, int unit_rays)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned u = 0;
        if (lane == 0) u = atomicAdd(queue + (NODES ? 1 : 0), 1u);
        u = __builtin_amdgcn_readfirstlane(__shfl(u, 0, 64));
        if (u >= n_units) break;
        const int64_t ray0 = (int64_t)u * unit_rays;  // state index of the unit's first ray
        const int k = __builtin_amdgcn_readfirstlane(find_segment(segs, nseg, ray0 >> 8));
        const BatchSeg sg = segs[k];
        const TraceParams &P = params[sg.image];
        if ((P.node_layout != 0) != NODES) continue;  // the other kernel's image
        for (int sub = 0; sub < unit_rays; sub += 64) {
            const int64_t idx = ray0 + sub + lane;
            if (idx - sg.slot_base * 256 >= sg.n_rays) continue;
            RayState r = st[idx];
            if ((r.info & (RS_ENTERED | RS_SURR)) != RS_ENTERED) continue;
            box_ray<float, NODES>(P, r);
            st[idx] = r;
        }
    }
}

template <int TILE>
__global__ void __launch_bounds__(256) k_finish_batch(const TraceParams *__restrict__ params,
                                                      const BatchSeg *__restrict__ segs, int nseg,
                                                      const RayState *__restrict__ st)
{
    __shared__ FinishShared<TILE> sh;
    if (threadIdx.x < CNT_SLOTS) sh.cnt[threadIdx.x] = 0ull;
    const int k = __builtin_amdgcn_readfirstlane(find_segment(segs, nseg, blockIdx.x));
    const BatchSeg sg = segs[k];
    const TraceParams &P = params[sg.image];
    const int64_t base = (int64_t)(blockIdx.x - sg.slot_base) * 256;
    // states of this segment start at slot_base * 256; ray ids at first_ray
    finish_block<TILE>(P, st + sg.slot_base * 256, sg.first_ray, base, sg.n_rays, sh);
    flush_counters<TILE>(P, sh);
}

// ------------------------------------------------------------------ ray surrogate

// Entry point (world) and unit direction of an emitted state that entered through z = z_lo.
__device__ __forceinline__ bool entry_of(const TraceParams &P, const RayState &r, double E[3], double u[3])
{
    if (!(r.info & RS_ENTERED) || r.c[2] != 0 || r.fd[2] != 0.0) return false;
    double n2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        E[a] = P.origin[a] + ((double)r.c[a] + r.fd[a]) * P.spacing[a];
        u[a] = (double)r.Tr[a] + (double)r.dT[a];
        n2 += u[a] * u[a];
    }
    const double il = 1.0 / sqrt(n2);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] *= il;
    return u[2] > 0.0;
}

__device__ __forceinline__ void surr_features(const SurrogateSpec &sp, const double E[3], const double u[3], float x[6])
{
    x[0] = (float)((2.0 * E[0] - sp.x_lo - sp.x_hi) * sp.inv_wx);
    x[1] = (float)((2.0 * E[1] - sp.y_lo - sp.y_hi) * sp.inv_wy);
    x[2] = (float)(u[0] * sp.inv_theta);
    x[3] = (float)(u[1] * sp.inv_theta);
    // the periodic encodings in single precision (inputs of an FP32 layer)
    x[4] = sinf((float)((E[0] - sp.x_lo) * sp.kx));
    x[5] = sinf((float)((E[1] - sp.y_lo) * sp.ky));
}

__device__ __forceinline__ int surr_tile(const SurrogateSpec &sp, const double E[3])
{
    int tx = (int)((E[0] - sp.x_lo) * sp.inv_wx * sp.tiles);
    int ty = (int)((E[1] - sp.y_lo) * sp.inv_wy * sp.tiles);
    tx = min(max(tx, 0), sp.tiles - 1);
    ty = min(max(ty, 0), sp.tiles - 1);
    return ty * sp.tiles + tx;
}

// Straight-line exit on z = z_hi from the entry.
__device__ __forceinline__ void straight_exit(const SurrogateSpec &sp, const double E[3], const double u[3], double Q[3])
{
    const double l = (sp.z_hi - E[2]) / u[2];
    Q[0] = E[0] + l * u[0];
    Q[1] = E[1] + l * u[1];
    Q[2] = sp.z_hi;
}

__global__ void __launch_bounds__(256) k_surr_samples(TraceParams P, SurrogateSpec sp, const RayState *__restrict__ st,
                                                      int64_t first, int64_t n, SurrogateSample *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    SurrogateSample smp;
    for (int k = 0; k < 6; ++k) smp.t[k] = 0.0f;
    smp.E[0] = smp.E[1] = 0.0; smp.u[0] = smp.u[1] = smp.u[2] = 0.0; smp.px[0] = smp.px[1] = 0.0;
    smp.tile = 0;
    smp.flags = 0;
    RayState e;
    emit_ray(P, ray_key(P, first + i), e);  // the entry state again (the trace overwrote it)
    double E[3], u[3];
    const RayState r = st[i];
    const bool enters = entry_of(P, e, E, u);
    if (enters) {
        smp.E[0] = E[0];
        smp.E[1] = E[1];
        smp.tile = surr_tile(sp, E);
        smp.flags = 4;
    }
    if (enters && !(r.info & RS_LIMITED) && r.c[2] == P.nz - 2 && r.fd[2] == 1.0) {
        double X[3], d[3], Q[3], n2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            X[a] = P.origin[a] + ((double)r.c[a] + r.fd[a]) * P.spacing[a];
            d[a] = (double)r.Tr[a] + (double)r.dT[a];
            n2 += d[a] * d[a];
        }
        const double il = 1.0 / sqrt(n2);
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] *= il;
        straight_exit(sp, E, u, Q);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            smp.t[a] = (float)(X[a] - Q[a]);
            smp.t[3 + a] = (float)(d[a] - u[a]);
            smp.u[a] = u[a];
        }
        smp.flags |= 1;
        double xp, yp;
        if (optics_to_sensor(P, X, d, &xp, &yp) == PBR_RAY_DEPOSITED) {
            smp.px[0] = xp;
            smp.px[1] = yp;
            smp.flags |= 2;
        }
    }
    out[i] = smp;
}

// Features of every ray of the chunk in place (row i = ray i; rows of rays the network does not
// take are zero and flagged 0 in elig), and the list of the other rays that entered the box for
// the integration kernel (one atomic per wave that has any).
__global__ void __launch_bounds__(256) k_surr_features(TraceParams P, SurrogateSpec sp, const RayState *__restrict__ st,
                                                       int64_t n, float *__restrict__ x,
                                                       unsigned char *__restrict__ elig, int *__restrict__ tlist,
                                                       unsigned long long *__restrict__ tcount)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    double E[3], u[3];
    bool ok = false, traced = false;
    if (i < n) {
        const RayState r = st[i];
        ok = entry_of(P, r, E, u);
        if (ok) ok = sp.tile_ok[surr_tile(sp, E)] != 0;
        traced = !ok && (r.info & RS_ENTERED);
        float f[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (ok) surr_features(sp, E, u, f);
#pragma unroll
        for (int k = 0; k < 6; ++k) x[i * 6 + k] = f[k];
        elig[i] = ok ? 1 : 0;
    }
    const unsigned long long tmask = __ballot(traced);
    if (tmask) {
        unsigned long long tbase = 0;
        if (lane == 0) tbase = atomicAdd(tcount, (unsigned long long)__popcll(tmask));
        tbase = __shfl(tbase, 0);
        if (traced) tlist[tbase + __popcll(tmask & ((1ull << lane) - 1ull))] = (int)i;
    }
}

// Predicted exit: straight exit plus the position change (on z = z_hi), direction u + change.
__device__ __forceinline__ void surr_predict(const SurrogateSpec &sp, const double E[3], const double u[3],
                                             const float *y, double X[3], double d[3])
{
    double Q[3];
    straight_exit(sp, E, u, Q);
    double n2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double dp = (double)y[a] * sp.t_scale[a] + sp.t_mean[a];
        const double dd = (double)y[3 + a] * sp.t_scale[3 + a] + sp.t_mean[3 + a];
        X[a] = Q[a] + dp;
        d[a] = u[a] + dd;
        n2 += d[a] * d[a];
    }
    X[2] = sp.z_hi;
    const double il = 1.0 / sqrt(n2);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= il;
}

__global__ void __launch_bounds__(256) k_surr_apply(TraceParams P, SurrogateSpec sp, const float *__restrict__ y,
                                                    const unsigned char *__restrict__ elig, int64_t n,
                                                    RayState *__restrict__ st)
{
    __shared__ unsigned s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && elig[i]) {
        RayState r = st[i];
        double E[3], u[3], X[3], d[3];
        entry_of(P, r, E, u);
        surr_predict(sp, E, u, y + i * 6, X, d);
        const int nn[3] = {P.nx, P.ny, P.nz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double p = (X[a] - P.origin[a]) / P.spacing[a];
            if (a == 2) p = (double)(nn[2] - 1);
            p = p < 0.0 ? 0.0 : (p > (double)(nn[a] - 1) ? (double)(nn[a] - 1) : p);
            int ci = (int)floor(p);
            ci = ci > nn[a] - 2 ? nn[a] - 2 : ci;
            r.c[a] = ci;
            r.fd[a] = p - (double)ci;
            r.Tr[a] = (float)d[a];
            r.dT[a] = (float)(d[a] - (double)r.Tr[a]);
        }
        r.info = RS_ENTERED | RS_SURR;
        st[i] = r;
        atomicAdd(&s_cnt, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomic_add_u64(P.counters + CNT_SURR, (unsigned long long)s_cnt);
}

__global__ void __launch_bounds__(256) k_surr_validate(TraceParams P, SurrogateSpec sp,
                                                       const SurrogateSample *__restrict__ smp, const float *__restrict__ y,
                                                       int64_t n, float *__restrict__ err, unsigned *__restrict__ tile_err,
                                                       unsigned *__restrict__ tile_cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const SurrogateSample s = smp[i];
    float e = -1.0f;  // not compared
    if ((s.flags & 5) == 4) {
        // entered through the front face but left elsewhere: the network cannot represent it
        e = 1.0e30f;
    } else if (s.flags & 1) {
        const double E[3] = {s.E[0], s.E[1], sp.z_lo};
        double X[3], d[3], xp, yp;
        surr_predict(sp, E, s.u, y + i * 6, X, d);
        const bool dep = optics_to_sensor(P, X, d, &xp, &yp) == PBR_RAY_DEPOSITED;
        if (dep && (s.flags & 2))
            e = (float)sqrt((xp - s.px[0]) * (xp - s.px[0]) + (yp - s.px[1]) * (yp - s.px[1]));
        else if (dep != ((s.flags & 2) != 0))
            e = -2.0f;  // passes an aperture or lens rim on one side and not the other
    }
    // a rim case would add or drop a whole ray: its tile is never eligible (the tracer keeps it)
    const float te = e == -2.0f ? 1.0e30f : e;
    if (te >= 0.0f) {
        atomicMax(tile_err + s.tile, __float_as_uint(te));
        atomicAdd(tile_cnt + s.tile, 1u);
    }
    err[i] = e;
}

__global__ void __launch_bounds__(256) k_surr_gather(SurrogateSpec sp, const SurrogateSample *__restrict__ smp,
                                                     const int *__restrict__ idx, int64_t rows, float *__restrict__ x,
                                                     float *__restrict__ t, const int *__restrict__ step,
                                                     int64_t steps_per_epoch)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * 6) return;
    if (step) idx += (int64_t)(*step % steps_per_epoch) * rows;
    const int64_t m = q / 6;
    const int k = (int)(q % 6);
    const SurrogateSample &s = smp[idx ? (int64_t)idx[m] : m];
    const double E[3] = {s.E[0], s.E[1], sp.z_lo};
    float f[6];
    surr_features(sp, E, s.u, f);
    x[q] = f[k];
    t[q] = (s.t[k] - sp.t_mean[k]) / sp.t_scale[k];
}

__global__ void __launch_bounds__(256) k_surr_moments(const SurrogateSample *__restrict__ smp, int64_t n,
                                                      double *__restrict__ part)
{
    __shared__ double s[kMoments][256];
    double a[kMoments];
#pragma unroll
    for (int k = 0; k < kMoments; ++k) a[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const SurrogateSample &q = smp[i];
        if (!(q.flags & 1)) continue;
        a[0] += 1.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double v = q.t[k];
            a[1 + k] += v;
            a[7 + k] += v * v;
        }
        a[13] += q.u[0] * q.u[0];
        a[14] += q.u[1] * q.u[1];
    }
#pragma unroll
    for (int k = 0; k < kMoments; ++k) s[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int k = 0; k < kMoments; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < kMoments) part[blockIdx.x * kMoments + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_surr_extract(const SurrogateSample *__restrict__ smp, int64_t n, int field,
                                                      int *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = field ? smp[i].tile : smp[i].flags;
}

}  // namespace

int launch_surr_extract(const SurrogateSample *smp, int64_t n, int field, int *out, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_surr_extract, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, smp, n, field, out);
    return (int)hipGetLastError();
}

int launch_surr_samples(const TraceParams &p, const SurrogateSpec &sp, const RayState *st, int64_t first,
                        int64_t n, SurrogateSample *out, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_surr_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, sp, st, first, n, out);
    return (int)hipGetLastError();
}

int launch_surr_features(const TraceParams &p, const SurrogateSpec &sp, const RayState *st, int64_t n, float *x,
                         unsigned char *elig, int *tlist, unsigned long long *tcount, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_surr_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, sp, st, n, x, elig,
                       tlist, tcount);
    return (int)hipGetLastError();
}

int launch_surr_apply(const TraceParams &p, const SurrogateSpec &sp, const float *y, const unsigned char *elig,
                      int64_t n, RayState *st, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_surr_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, sp, y, elig, n, st);
    return (int)hipGetLastError();
}

int launch_surr_validate(const TraceParams &p, const SurrogateSpec &sp, const SurrogateSample *smp,
                         const float *y, int64_t n, float *err, unsigned *tile_err, unsigned *tile_cnt,
                         hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_surr_validate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, sp, smp, y, n, err,
                       tile_err, tile_cnt);
    return (int)hipGetLastError();
}

int launch_surr_gather(const SurrogateSpec &sp, const SurrogateSample *smp, const int *idx, int64_t rows,
                       float *x, float *t, hipStream_t s)
{
    if (rows <= 0) return 0;
    hipLaunchKernelGGL(k_surr_gather, dim3((unsigned)((rows * 6 + 255) / 256)), dim3(256), 0, s, sp, smp, idx, rows,
                       x, t, (const int *)nullptr, (int64_t)1);
    return (int)hipGetLastError();
}

int launch_surr_gather_step(const SurrogateSpec &sp, const SurrogateSample *smp, const int *perm, const int *step,
                            int64_t steps_per_epoch, int64_t rows, float *x, float *t, hipStream_t s)
{
    hipLaunchKernelGGL(k_surr_gather, dim3((unsigned)((rows * 6 + 255) / 256)), dim3(256), 0, s, sp, smp, perm, rows,
                       x, t, step, steps_per_epoch);
    return (int)hipGetLastError();
}

int launch_surr_moments(const SurrogateSample *smp, int64_t n, double *part, int *blocks, hipStream_t s)
{
    int nb = (int)((n + 255) / 256);
    nb = nb < 1024 ? (nb < 1 ? 1 : nb) : 1024;
    *blocks = nb;
    hipLaunchKernelGGL(k_surr_moments, dim3((unsigned)nb), dim3(256), 0, s, smp, n, part);
    return (int)hipGetLastError();
}

int launch_calibrate(const TraceParams &p, const int *bricks, int n_bricks, int rays_per_brick,
                     int n_steps, uint64_t seed, double z_focus, double px_per_m, float *err,
                     hipStream_t stream)
{
    if (n_bricks <= 0) return 0;
    if (p.node_layout)
        hipLaunchKernelGGL(k_calibrate<true>, dim3((unsigned)n_bricks), dim3((unsigned)rays_per_brick), 0, stream, p,
                           bricks, n_steps, seed, z_focus, px_per_m, err);
    else
        hipLaunchKernelGGL(k_calibrate<false>, dim3((unsigned)n_bricks), dim3((unsigned)rays_per_brick), 0, stream, p,
                           bricks, n_steps, seed, z_focus, px_per_m, err);
    return (int)hipGetLastError();
}

int launch_trace_chunk(const TraceParams &p, RayState *st, int64_t first, int64_t n, int prec,
                       hipStream_t stream, hipEvent_t box_begin, hipEvent_t box_end, const ChunkHook *hook,
                       bool deposit, bool refill)
{
    if (n <= 0) return 0;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(256), 0, stream, p, st, first, n);
    int e = (int)hipGetLastError();
    if (e) return e;
    TraceList tl{nullptr, nullptr};
    if (hook && (e = hook->run(hook->self, p, st, first, n, stream, &tl))) return e;
    if (box_begin && (e = (int)hipEventRecord(box_begin, stream))) return e;
    if (prec == PREC_FP64) {
        if (p.node_layout) hipLaunchKernelGGL(k_box64<true>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
        else hipLaunchKernelGGL(k_box64<false>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
    }
    else if (prec == PREC_MIXED) {
        if (p.node_layout) hipLaunchKernelGGL(k_box_mixed<true>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
        else hipLaunchKernelGGL(k_box_mixed<false>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
    }
    else if (refill) {
        // persistent grid: five 256-thread blocks per compute unit, fewer for small chunks
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        const unsigned pblocks = (unsigned)ncu * 5u < blocks ? (unsigned)ncu * 5u : blocks;
        if ((e = launch_clear_u64(p.counters + CNT_QUEUE, 1, stream))) return e;
        hipLaunchKernelGGL(k_box32_refill, dim3(pblocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count,
                           p.counters + CNT_QUEUE);
    } else if (p.node_layout)
        hipLaunchKernelGGL(k_box32<true>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
    else
        hipLaunchKernelGGL(k_box32<false>, dim3(blocks), dim3(256), 0, stream, p, st, n, tl.idx, tl.count);
    e = (int)hipGetLastError();
    if (e) return e;
    if (box_end && (e = (int)hipEventRecord(box_end, stream))) return e;
    if (!deposit) return 0;
    unsigned fblocks = blocks < 4096u ? blocks : 4096u;
    const RayState *cst = st;
    const int feat = (p.mie ? FEAT_MIE : 0) | (p.chain ? FEAT_CHAIN : 0);
    if (feat) {
        // spot radii of 1-3 pixels cover focused particles; wider spots take the run-time radius
        const int rf = p.rfp <= 3 ? p.rfp : 0;
#define PBR_FINISH_FEAT(F)                                                                                          \
        switch (rf) {                                                                                               \
            case 1: hipLaunchKernelGGL((k_finish<kTile, 1, F>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break; \
            case 2: hipLaunchKernelGGL((k_finish<kTile, 2, F>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break; \
            case 3: hipLaunchKernelGGL((k_finish<kTile, 3, F>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break; \
            default: hipLaunchKernelGGL((k_finish<kTile, 0, F>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break; \
        }
        if (feat == FEAT_MIE) { PBR_FINISH_FEAT(FEAT_MIE) }
        else if (feat == FEAT_CHAIN) { PBR_FINISH_FEAT(FEAT_CHAIN) }
        else { PBR_FINISH_FEAT(FEAT_MIE | FEAT_CHAIN) }
#undef PBR_FINISH_FEAT
    }
    else switch (p.rfp) {
        case 1: hipLaunchKernelGGL((k_finish<kTile, 1>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 2: hipLaunchKernelGGL((k_finish<kTile, 2>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 3: hipLaunchKernelGGL((k_finish<kTile, 3>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 4: hipLaunchKernelGGL((k_finish<kTile, 4>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 5: hipLaunchKernelGGL((k_finish<kTile, 5>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 6: hipLaunchKernelGGL((k_finish<kTile, 6>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        case 7: hipLaunchKernelGGL((k_finish<kTile, 7>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
        default: hipLaunchKernelGGL((k_finish<kTile, 8>), dim3(fblocks), dim3(256), 0, stream, p, cst, first, n); break;
    }
    return (int)hipGetLastError();
}

int launch_batch_round(const TraceParams *params, const BatchSeg *segs, int nseg, int64_t n_slots,
                       RayState *st, unsigned *queue, const BatchConfig &cfg, int n_cu, hipStream_t stream,
                       bool cells, bool nodes)
{
    if (n_slots <= 0) return 0;
    int e = launch_clear_u64((unsigned long long *)queue, 1, stream);  // both counters
    if (e) return e;
    hipLaunchKernelGGL(k_emit_batch, dim3((unsigned)n_slots), dim3(256), 0, stream, params, segs, nseg, st);
    if ((e = (int)hipGetLastError())) return e;
    const unsigned n_units = (unsigned)(n_slots * 256 / cfg.unit_rays);
    // a persistent grid per field layout present in the round: five waves per SIMD for the
    // per-cell kernel, four for the node kernel (its register budget)
    const unsigned w_cells = (unsigned)n_cu * 4u * 5u, w_nodes = (unsigned)n_cu * 4u * 4u;
    if (cells) {
        if (cfg.box_block == 64)
            hipLaunchKernelGGL((k_box_batch<64, false>), dim3(w_cells), dim3(64), 0, stream, params, segs, nseg, st,
                               queue, n_units, cfg.unit_rays);
        else
            hipLaunchKernelGGL((k_box_batch<256, false>), dim3(w_cells / 4u), dim3(256), 0, stream, params, segs,
                               nseg, st, queue, n_units, cfg.unit_rays);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (nodes) {
        if (cfg.box_block == 64)
            hipLaunchKernelGGL((k_box_batch<64, true>), dim3(w_nodes), dim3(64), 0, stream, params, segs, nseg, st,
                               queue, n_units, cfg.unit_rays);
        else
            hipLaunchKernelGGL((k_box_batch<256, true>), dim3(w_nodes / 4u), dim3(256), 0, stream, params, segs,
                               nseg, st, queue, n_units, cfg.unit_rays);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (cfg.tile == 16)
        hipLaunchKernelGGL(k_finish_batch<16>, dim3((unsigned)n_slots), dim3(256), 0, stream, params, segs, nseg,
                           (const RayState *)st);
    else
        hipLaunchKernelGGL(k_finish_batch<32>, dim3((unsigned)n_slots), dim3(256), 0, stream, params, segs, nseg,
                           (const RayState *)st);
    return (int)hipGetLastError();
}

}  // namespace pbr
