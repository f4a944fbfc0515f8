// rtm.hip -- HIP kernels for gfx950 and the extern "C" entry points of librtm.so.
//
// The per-time-step phases follow the paper's section II (halo stencil, pack, exchange, interior
// stencil, unpack); the scheme is the radius-R star stencil with second-order leapfrog and a
// Cerjan sponge:  u^{n+1} = g (2 u^n - g u^{n-1} + kappa L u^n).
//
// Every stencil kernel evaluates the same per-point expression (point_op) on the same operands
// in the same order, with explicit FMAs and FP contraction disabled at compile time, so any split of
// a step between the halo and interior calls produces bitwise identical wavefields.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <utility>

#include "rtm.h"

namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------------------------
// Device-side geometry (passed by value to every kernel)
// ---------------------------------------------------------------------------------------------
struct Geo {
    int nx, ny, nz, R;
    long long py, pz;
    float c[5];
    const float *gx, *gy, *gz;
};

__device__ __forceinline__ long long pidx(const Geo &g, int i, int j, int k)
{
    return (long long)(k + g.R) * g.pz + (long long)(j + g.R) * g.py + (long long)(i + g.R);
}

// Sum of the six neighbours at distance m: ((x- + x+) + (y- + y+)) + (z- + z+).
__device__ __forceinline__ float axis_sum(float xm, float xp, float ym, float yp, float zm, float zp)
{
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// What a stencil kernel computes at a cell from the stencil field u (its Laplacian lap), two
// centre operands a, b and the sponge factor g:
//   OP_FORWARD   u = u^n,            a = u^{n-1}, b = kappa:   g (2 u^n - g u^{n-1} + kappa L u^n)
//   OP_ADJOINT   u = kappa g mu_a,   a = mu_a,    b = mu_b:    2 g mu_a + L(kappa g mu_a) - g^2 mu_b
//                (the tiled kernel forms u itself from mu_a and kappa as it loads each plane)
//   OP_GRADIENT  u = u^n,            a = mu,      b = grad:    grad + g mu L u^n
//   OP_GRADIENT_SCALED u = u^n,      a = w,       b = grad:    grad + w L u^n   (w = kappa g mu)
enum { OP_FORWARD = 0, OP_ADJOINT = 1, OP_GRADIENT = 2, OP_GRADIENT_SCALED = 3 };

// The per-point operation.  s[m-1] = axis_sum at distance m.  The centre weight is 3 c0 (one c0 per
// axis).
template <int R, int OP>
__device__ __forceinline__ float point_op(float u0, const float (&s)[R], float a, float b, float g,
                                          const float (&c)[5])
{
    float lap = (3.0f * c[0]) * u0;
#pragma unroll
    for (int m = 1; m <= R; ++m)
        lap = __builtin_fmaf(c[m], s[m - 1], lap);
    if constexpr (OP == OP_FORWARD) {
        float t = __builtin_fmaf(-g, a, 2.0f * u0);
        t = __builtin_fmaf(b, lap, t);
        return g * t;
    } else if constexpr (OP == OP_ADJOINT) {
        const float t = __builtin_fmaf(2.0f * g, a, lap);
        return __builtin_fmaf(-(g * g), b, t);
    } else if constexpr (OP == OP_GRADIENT) {
        return __builtin_fmaf(g * a, lap, b);
    } else {
        return __builtin_fmaf(a, lap, b);
    }
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }

// Non-temporal (streaming) forms, for data used once per step (u^{n-1}, kappa, u^{n+1}).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4_nt(const float *p)
{
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4_nt(float *p, float4 v)
{
    const f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f4v *>(p));
}

// Cross-lane moves of a float4 by one lane (DPP wave_shr:1 / wave_shl:1): lane l receives lane l - 1's
// (shr) or lane l + 1's (shl) value; the lane with no source receives 0.  Every lane of the wave must
// be active.
__device__ __forceinline__ float dpp_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float4 dpp_shr1(float4 v) { return make_float4(dpp_shr1(v.x), dpp_shr1(v.y), dpp_shr1(v.z), dpp_shr1(v.w)); }
__device__ __forceinline__ float4 dpp_shl1(float4 v) { return make_float4(dpp_shl1(v.x), dpp_shl1(v.y), dpp_shl1(v.z), dpp_shl1(v.w)); }

// Variants of the tiled kernel (template flags): streaming hints on the once-used streams, the
// x neighbours of a thread's float4 taken from the adjacent lanes' registers instead of LDS, (radius-4
// forward launches) the ghost cells of u_cur read from the receive slots instead of the ghost ring, and
// (the shell call) the computed cells written to the face buffer only, not to u_nxt.
enum { FL_NT = 1, FL_XSHUF = 2, FL_SLOTS = 4, FL_PONLY = 8 };
__device__ __forceinline__ float el(const float4 &v, int e)
{
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

__device__ __forceinline__ float sponge(const Geo &g, int i, int j, int k)
{
    return (g.gx[i] * g.gy[j]) * g.gz[k];
}

// Scalar update of one owned cell, reading every operand from global memory.
template <int R, int OP>
__device__ __forceinline__ void update_cell(const Geo &g, float *un, const float *uc, const float *up,
                                            const float *kap, int i, int j, int k)
{
    const long long p = pidx(g, i, j, k);
    const float u0 = uc[p];
    float s[R];
#pragma unroll
    for (int m = 1; m <= R; ++m)
        s[m - 1] = axis_sum(uc[p - m], uc[p + m], uc[p - m * g.py], uc[p + m * g.py], uc[p - m * g.pz],
                            uc[p + m * g.pz]);
    float c[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) c[m] = g.c[m];
    un[p] = point_op<R, OP>(u0, s, up[p], kap[p], sponge(g, i, j, k), c);
}

// ---------------------------------------------------------------------------------------------
// Halo shell: the owned cells within R of a face, as six slabs (-Z, +Z, -Y, +Y, -X, +X) that do
// not overlap.  blockIdx.y selects the slab; x is fastest inside a slab.
// ---------------------------------------------------------------------------------------------
struct Slab {
    int ox, oy, oz;   // origin (owned coordinates)
    int wx, wy, wz;   // extent
};

// Elementwise kernels walk their items with a grid-sized stride and 64-bit counters, so a launch of
// at most kMaxBlocks workgroups covers fields of more than 2^32 cells (one HIP launch dimension
// holds fewer than 2^32 work-items); below kMaxBlocks * kThreads items every thread takes one item.
__device__ __forceinline__ long long first_item() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long item_stride() { return (long long)gridDim.x * blockDim.x; }

// Scalar update over one box [x0,x1) x [y0,y1) x [z0,z1) (fallback for layouts the vectorised
// kernel cannot take).
template <int R, int OP>
__global__ __launch_bounds__(kThreads) void k_box(Geo g, float *un, const float *__restrict__ uc, const float *up,
                                                  const float *kap, int x0, int x1, int y0, int y1, int z0, int z1)
{
    const long long wx = x1 - x0, wy = y1 - y0, wz = z1 - z0;
    for (long long t = first_item(); t < wx * wy * wz; t += item_stride()) {
        const int i = x0 + (int)(t % wx);
        const int j = y0 + (int)((t / wx) % wy);
        const int k = z0 + (int)(t / (wx * wy));
        update_cell<R, OP>(g, un, uc, up, kap, i, j, k);
    }
}

// ---------------------------------------------------------------------------------------------
// Interior: 2.5-D blocking (Micikevicius 2009) for CDNA4.
//
// A workgroup of BX x BY threads owns an XY tile of TX = 4 BX columns by TY = BY rows and marches
// through a chunk of z planes.  Each thread owns four consecutive x cells (one float4) of one row:
//   * z neighbours come from a register queue of 2R+1 float4 planes that shifts by one each step;
//   * x and y neighbours come from the current plane, staged with a 4-column / R-row halo in LDS
//     (double-buffered, so one barrier per plane);
//   * the next plane's loads are issued before the current plane is computed.
// Workgroup ids are remapped so that each of the 8 XCDs (round-robin dispatch) receives a
// contiguous range of tiles, keeping the halo re-reads of neighbouring tiles in the same L2.
// ---------------------------------------------------------------------------------------------

// Calls f(integral_constant<int, I>) for I = 0, 1, ... in order while it returns true, with I a
// compile-time constant in every call (so arrays indexed by it stay in registers).
template <typename F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>)
{
    (void)(f(std::integral_constant<int, I>{}) && ...);
}

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int xcd = b & 7, q = nb >> 3, r = nb & 7;
    return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

struct Box {
    int x0, x1, y0, y1, z0, z1;   // owned-cell bounds of the box
    int X0;                       // first tile column: x0 aligned down so that X0 + R is a multiple of 4
    int zchunk, ntx, nty, nzc;
    int nblk;                     // ntx * nty * nzc
};

constexpr int kMaxBoxes = 6;

struct BoxList {
    Box b[kMaxBoxes];
    int nbox;
    int nblk;     // sum of the boxes' nblk
    int remap;
};

// Where a halo launch with PACK also writes the face cells it computes: the face buffer and the six
// slot offsets of rtm_face_layout.
// With FL_SLOTS, recv[f] is the receive slot of ghost face f (the layout rtm_unpack_halo reads).
struct PackOut {
    float *faces;
    long long off[6];
    const float *recv[6];
};

// kappa g mu for the four cells of a float4, in the order (kappa (gxy gz)) mu, and exactly zero for
// the cells whose bit in `in` is clear (cells outside the owned block: their values are never read).
__device__ __forceinline__ float4 weight4(float4 mu, float4 kp, const float (&gxy)[4], float gz, unsigned in)
{
    float4 w;
    w.x = (in & 1u) ? (kp.x * (gxy[0] * gz)) * mu.x : 0.0f;
    w.y = (in & 2u) ? (kp.y * (gxy[1] * gz)) * mu.y : 0.0f;
    w.z = (in & 4u) ? (kp.z * (gxy[2] * gz)) * mu.z : 0.0f;
    w.w = (in & 8u) ? (kp.w * (gxy[3] * gz)) * mu.w : 0.0f;
    return w;
}

// LDS of one tile: R + 2 planes of (BY + 2R) rows of BX + 2 float4s.
template <int R, int BX, int BY>
struct TileLds {
    static constexpr int S = R + 2, LH = BY + 2 * R, LW4 = BX + 2, N = S * LH * LW4;
};

// One workgroup of the tiled kernel: block `bid` of the box list, its LDS at `lds_raw`
// (TileLds<R, BX, BY>::N float4s).  The structs come by value, as kernel arguments do.
template <int R, int BX, int BY, int OP, bool PACK, int FL>
__device__ __forceinline__ void tiled_body(int bid, float4 *lds_raw, const Geo g, float *un,
                                           const float *__restrict__ uc, const float *up, const float *kap,
                                           const BoxList bl, const PackOut po, const float *__restrict__ rk)
{
    constexpr bool STREAM = (FL & FL_NT) != 0;
    constexpr bool XS = (FL & FL_XSHUF) != 0;
    constexpr bool GS = (FL & FL_SLOTS) != 0;
    constexpr bool PONLY = (FL & FL_PONLY) != 0;
    auto ldo = [](const float *p) { return STREAM ? ld4_nt(p) : ld4(p); };   // u_prv / kappa operands
    // OP_ADJOINT: the stencil field is kappa g mu_a, formed here from two loads per ring element (uc =
    // mu_a, rk = kappa) instead of being read from a field written by a separate pass; the ring
    // elements of cells outside the owned block are zero, as the ghosts of such a field would be.
    constexpr bool WR = (OP == OP_ADJOINT);
    static_assert(!GS || (R == 4 && !WR), "ghosts from slots: radius-4 forward launches only");
    static_assert(!PONLY || (PACK && GS), "face buffer only: the shell call");
    constexpr int NT = BX * BY;
    constexpr int TX = 4 * BX;
    constexpr int TY = BY;
    constexpr int LW4 = BX + 2;            // LDS row in float4: 1 halo, BX centre, 1 halo
    constexpr int LH = TY + 2 * R;         // LDS rows: R halo rows above and below
    constexpr int NH = 2 * R * BX + 2 * BY; // halo float4 items per plane
    constexpr int HPT = (NH + NT - 1) / NT;
    constexpr int QR = 2 * R + 2;          // register ring: the 2R+1 planes in use plus the one in flight
    constexpr int S = R + 2;               // LDS ring: planes k-1 .. k+R
    static_assert(TileLds<R, BX, BY>::N == S * LH * LW4, "LDS size");
    auto &lds = *reinterpret_cast<float4 (*)[S][LH][LW4]>(lds_raw);

    int lb = bl.remap ? xcd_remap(bid, bl.nblk) : bid;
    Box bx = bl.b[0];
#pragma unroll
    for (int i = 1; i < kMaxBoxes; ++i) {
        if (i < bl.nbox && lb >= bx.nblk) {
            lb -= bx.nblk;
            bx = bl.b[i];
        }
    }
    const int tix = lb % bx.ntx;
    const int tiy = (lb / bx.ntx) % bx.nty;
    const int tiz = lb / (bx.ntx * bx.nty);
    const int X = bx.X0 + tix * TX;
    const int Y = bx.y0 + tiy * TY;
    const int zs = bx.z0 + tiz * bx.zchunk;
    const int ze = min(zs + bx.zchunk, bx.z1);

    const int tid = threadIdx.x;
    const int lx = tid % BX, ly = tid / BX;
    const int x = X + 4 * lx, y = Y + ly;
    const int xlim = bx.x1 + R;            // columns >= xlim are never needed
    const int ylim = bx.y1 + R;
    const int elo = max(0, bx.x0 - x);     // cells of this float4 before the box
    const int ehi = min(4, bx.x1 - x);     // cells of this float4 inside the box end here
    const bool active = (ehi > elo) && (y < bx.y1);
    const bool full = active && elo == 0 && ehi == 4;
    const bool cload = (x < xlim) && (y < ylim);
    const long long pz = g.pz;

    // centre column pointer at plane zs.  Lanes whose column or row is not needed load from the
    // tile origin instead (always inside the padded block), so every load is unconditional; what
    // they load is never read.
    const long long pc = pidx(g, x, y, zs);
    const long long p0 = pidx(g, X, Y, zs);
    const long long pcl = cload ? pc : p0;
    const long long pca = active ? pc : p0;

    // GS: where a float4 of u_cur at column xx, row yy lives, as a pointer at plane zs and a plane
    // stride: owned cells in uc, ghost cells in the receive slot of their face, float4s that are
    // ghosts in both x and y (no active cell reads them) at the tile origin.  With R = 4 and
    // nx % 4 == 0 no float4 mixes owned and ghost cells.
    auto where = [&](int xx, int yy, const float *&base, long long &stride) {
        const long long nx = g.nx, ny = g.ny;
        const bool xin = xx >= 0 && xx < g.nx, yin = yy >= 0 && yy < g.ny;
        if (xin && yin) {
            base = uc + pidx(g, xx, yy, zs);
            stride = pz;
        } else if (yin) {           // x ghost: slot 0 or 1, one float4 per row
            base = (xx < 0 ? po.recv[0] : po.recv[1]) + ((long long)zs * ny + yy) * R;
            stride = ny * R;
        } else if (xin) {           // y ghost: slot 2 or 3, R rows per plane
            base = (yy < 0 ? po.recv[2] + ((long long)zs * R + (yy + R)) * nx
                           : po.recv[3] + ((long long)zs * R + (yy - g.ny)) * nx) + xx;
            stride = R * nx;
        } else {
            base = uc + p0;
            stride = pz;
        }
    };
    // GS: the centre column's source on owned planes (cb, cs) and in the z ghost slots (planes -R ..
    // -1 in slot 4, nz .. nz + R - 1 in slot 5; zst = 0 for a column that is not owned)
    const float *cb = uc + pcl, *zlo = uc + p0, *zhi = uc + p0;
    long long cs = pz, zst = 0;
    if constexpr (GS) {
        if (cload) where(x, y, cb, cs);
        if (cload && x < g.nx && y < g.ny) {
            const long long o = (long long)y * g.nx + x;
            zlo = po.recv[4] + o;
            zhi = po.recv[5] + o;
            zst = (long long)g.nx * g.ny;
        }
    }
    auto ldc = [&](int p) -> float4 {       // GS: centre column at plane p (uniform over the block)
        if (p < 0) return ld4(zlo + (long long)(p + R) * zst);
        if (p >= g.nz) return ld4(zhi + (long long)(p - g.nz) * zst);
        return ld4(cb + (long long)(p - zs) * cs);
    };

    // halo items owned by this thread: global offset at plane zs and LDS slot (row, float4 column)
    long long hoff[HPT];
    int hrow[HPT], hcol[HPT];
    bool hok[HPT];
    int hxx[HPT], hyy[HPT];
    const float *hb[HPT];                   // GS: the item's source at plane zs and its plane stride
    long long hs[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
        const int t = tid + h * NT;
        hok[h] = false;
        hoff[h] = p0;
        hrow[h] = 0;
        hcol[h] = 0;
        hxx[h] = X;
        hyy[h] = Y;
        if (t < 2 * R * BX) {
            const int yr = t / BX, col = t % BX;
            const int row = yr < R ? Y - R + yr : Y + TY + (yr - R);
            const int xx = X + 4 * col;
            hrow[h] = yr < R ? yr : TY + yr;
            hcol[h] = 1 + col;
            hok[h] = (xx < xlim) && (row < ylim);
            hoff[h] = hok[h] ? pidx(g, xx, row, zs) : p0;
            hxx[h] = xx;
            hyy[h] = row;
        } else if (t < NH) {
            const int t2 = t - 2 * R * BX;
            const int side = t2 / BY, r = t2 % BY;
            const int row = Y + r;
            const int xx = side == 0 ? X - 4 : X + TX;
            hrow[h] = R + r;
            hcol[h] = side == 0 ? 0 : 1 + BX;
            hok[h] = (side == 0 ? (X - 1 >= bx.x0 - R) : (xx < xlim)) && (row < ylim);
            hoff[h] = hok[h] ? pidx(g, xx, row, zs) : p0;
            hxx[h] = xx;
            hyy[h] = row;
        }
        hb[h] = uc + hoff[h];
        hs[h] = pz;
        if constexpr (GS)
            if (hok[h]) where(hxx[h], hyy[h], hb[h], hs[h]);
    }
    // WR: the x-y sponge factors of each halo item's four cells and which of them are owned cells
    float hg[HPT][4];
    unsigned hin[HPT];
    if constexpr (WR) {
#pragma unroll
        for (int h = 0; h < HPT; ++h) {
            const int yi = min(max(hyy[h], 0), g.ny - 1);
            const bool yin = hok[h] && hyy[h] >= 0 && hyy[h] < g.ny;
            hin[h] = 0u;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int xe = hxx[h] + e;
                hg[h][e] = g.gx[min(max(xe, 0), g.nx - 1)] * g.gy[yi];
                if (yin && xe >= 0 && xe < g.nx) hin[h] |= 1u << e;
            }
        }
    }

    float c[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) c[m] = g.c[m];
    float gxy[4];
    unsigned cin = 0u;                      // WR: which cells of this thread's column are owned
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int xi = min(max(x + e, 0), g.nx - 1);
        const int yi = min(y, g.ny - 1);
        gxy[e] = g.gx[xi] * g.gy[yi];
        if (x + e >= 0 && x + e < g.nx && y < g.ny) cin |= 1u << e;
    }
    // WR: the z sponge factor of plane p and whether p is an owned plane
    auto gzp = [&](int p) { return g.gz[min(max(p, 0), g.nz - 1)]; };
    auto zin = [&](int p) { return (p >= 0 && p < g.nz) ? 0xfu : 0u; };

    // Two rings.  (1) Registers: this thread's float4 of plane p of u_cur lives in
    // q[(p - zs + R) % QR]; the z loop is unrolled by QR so every ring index is a compile-time
    // constant.  (2) LDS: plane p with its x/y halo lives in lds[(p - zs) % S].  Both are filled at
    // the leading edge (plane k + R while plane k is computed), so a tile reads its halo rows at the
    // same time as the neighbouring tiles read them as their own centre rows, while they are in L2.
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 q[QR];
    float4 qm = zero4, qk = zero4;          // WR: mu and kappa of the centre plane in flight
    if constexpr (WR) {
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) {
            const long long o = pcl + (long long)(m - R) * pz;
            q[m] = weight4(ld4(uc + o), ld4(rk + o), gxy, gzp(zs - R + m), cin & zin(zs - R + m));
        }
        qm = ld4(uc + pcl + (long long)R * pz);
        qk = ld4(rk + pcl + (long long)R * pz);
        q[2 * R] = zero4;
    } else if constexpr (GS) {
#pragma unroll
        for (int m = 0; m < 2 * R + 1; ++m) q[m] = ldc(zs - R + m);
    } else {
#pragma unroll
        for (int m = 0; m < 2 * R + 1; ++m) q[m] = ld4(uc + pcl + (long long)(m - R) * pz);
    }
    q[QR - 1] = zero4;
    // LDS planes zs .. zs+R-1 (those that exist)
    for (int d = 0; d < R && zs + d < ze; ++d) {
        float4 hv[HPT];
        if constexpr (WR) {
            const float gz = gzp(zs + d);
            const unsigned zm = zin(zs + d);
#pragma unroll
            for (int h = 0; h < HPT; ++h) {
                const long long o = hoff[h] + (long long)d * pz;
                hv[h] = weight4(ld4(uc + o), ld4(rk + o), hg[h], gz, hin[h] & zm);
            }
            const long long o = pcl + (long long)d * pz;
            lds[d][R + ly][1 + lx] = weight4(ld4(uc + o), ld4(rk + o), gxy, gz, cin & zm);
        } else if constexpr (GS) {
#pragma unroll
            for (int h = 0; h < HPT; ++h) hv[h] = ld4(hb[h] + (long long)d * hs[h]);
            lds[d][R + ly][1 + lx] = ld4(cb + (long long)d * cs);
        } else {
#pragma unroll
            for (int h = 0; h < HPT; ++h) hv[h] = ld4(uc + hoff[h] + (long long)d * pz);
            lds[d][R + ly][1 + lx] = ld4(uc + pcl + (long long)d * pz);
        }
#pragma unroll
        for (int h = 0; h < HPT; ++h)
            if (tid + h * NT < NH) lds[d][hrow[h]][hcol[h]] = hv[h];
    }
    // halo of plane zs + R (written in the first iteration); WR keeps mu in hv and kappa in hk
    float4 hv[HPT], hk[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
        if constexpr (GS)   // a chunk shorter than R + 1 planes never stages this plane: clamped into it
            hv[h] = ld4(hb[h] + (long long)(min(zs + R, ze - 1) - zs) * hs[h]);
        else
            hv[h] = ld4(uc + hoff[h] + (long long)R * pz);
        if constexpr (WR) hk[h] = ld4(rk + hoff[h] + (long long)R * pz);
    }
    // operands of plane k (u_prv, kappa and the z sponge factor) arrive one plane ahead, in the same
    // batch of loads, so waiting for them never waits for the loads issued for later planes
    float4 pv[2], kv[2];
    float gzv[2];
    pv[0] = ldo(up + pca);
    kv[0] = ldo(kap + pca);
    gzv[0] = g.gz[zs];

    int k0_ = zs;                           // first plane of the current ring revolution
    int sk = 0;                             // LDS slot of plane k
    // One plane of the march; `S_` is the compile-time position of plane k in the register ring.
    auto plane = [&](auto S_) -> bool {
        constexpr int s = decltype(S_)::value;
        const int k = k0_ + s;
        if (k >= ze) return false;
        const int b = s & 1;               // operand slot of plane k
        const long long dz = (long long)(k - zs) * pz;
        const int sw = (sk + R < S) ? sk + R : sk + R - S;   // LDS slot of plane k + R
        // WR: plane k + R of the ring, from the mu and kappa loaded during the previous plane
        float gzr = 0.0f;
        unsigned zmr = 0u;
        if constexpr (WR) {
            gzr = gzp(k + R);
            zmr = zin(k + R);
            q[(s + 2 * R) % QR] = weight4(qm, qk, gxy, gzr, cin & zmr);
        }
        // stage plane k + R (centre from the register ring, halo from the pending loads)
        if (k + R < ze) {
            lds[sw][R + ly][1 + lx] = q[(s + 2 * R) % QR];
#pragma unroll
            for (int h = 0; h < HPT; ++h) {
                if (tid + h * NT < NH) {
                    if constexpr (WR)
                        lds[sw][hrow[h]][hcol[h]] = weight4(hv[h], hk[h], hg[h], gzr, hin[h] & zmr);
                    else
                        lds[sw][hrow[h]][hcol[h]] = hv[h];
                }
            }
        }
        __syncthreads();

        // issue the loads of plane k + R + 1 (centre into the ring slot of plane k - R - 1, which
        // is no longer needed; its halo) and of u_prv / kappa at plane k + 1.  They are issued on
        // every plane, with the plane index clamped to the chunk at its end (those values are never
        // used), so the number of loads in flight is the same on every path and the waits before
        // the compute only cover the previous plane's loads.
        {
            const long long kn = min(k + 1, ze - 1) - zs;          // plane of u_prv / kappa
            const long long kh = min(k + R + 1, ze - 1) - zs;      // plane of the halo
            if constexpr (WR) {
                qm = ld4(uc + pcl + (kn + R) * pz);
                qk = ld4(rk + pcl + (kn + R) * pz);
#pragma unroll
                for (int h = 0; h < HPT; ++h) {
                    hv[h] = ld4(uc + hoff[h] + kh * pz);
                    hk[h] = ld4(rk + hoff[h] + kh * pz);
                }
            } else if constexpr (GS) {
                q[(s + 2 * R + 1) % QR] = ldc(zs + (int)kn + R);
#pragma unroll
                for (int h = 0; h < HPT; ++h) hv[h] = ld4(hb[h] + kh * hs[h]);
            } else {
                q[(s + 2 * R + 1) % QR] = ld4(uc + pcl + (kn + R) * pz);
#pragma unroll
                for (int h = 0; h < HPT; ++h) hv[h] = ld4(uc + hoff[h] + kh * pz);
            }
            pv[b ^ 1] = ldo(up + pca + kn * pz);
            kv[b ^ 1] = ldo(kap + pca + kn * pz);
            gzv[b ^ 1] = g.gz[zs + kn];
        }

        // XS: the neighbouring float4s of the row from the adjacent lanes (all lanes active here; lanes
        // of one row are consecutive), the tile's edge lanes from the LDS halo columns
        float4 xls = zero4, xrs = zero4;
        if constexpr (XS) {
            xls = dpp_shr1(q[(s + R) % QR]);
            xrs = dpp_shl1(q[(s + R) % QR]);
        }
        if (active) {
            const float4 xc = q[(s + R) % QR];
            float4 xl, xr;
            if constexpr (XS) {
                xl = xls;
                xr = xrs;
                if (lx == 0) xl = lds[sk][R + ly][0];
                if (lx == BX - 1) xr = lds[sk][R + ly][BX + 1];
            } else {
                xl = lds[sk][R + ly][lx];
                xr = lds[sk][R + ly][2 + lx];
            }
            float4 ym[R], yp[R];
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                ym[m - 1] = lds[sk][R + ly - m][1 + lx];
                yp[m - 1] = lds[sk][R + ly + m][1 + lx];
            }
            const float xs[12] = {xl.x, xl.y, xl.z, xl.w, xc.x, xc.y, xc.z, xc.w, xr.x, xr.y, xr.z, xr.w};
            const float gz = gzv[b];
            float out[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float sm[R];
#pragma unroll
                for (int m = 1; m <= R; ++m)
                    sm[m - 1] = axis_sum(xs[4 + e - m], xs[4 + e + m], el(ym[m - 1], e), el(yp[m - 1], e),
                                         el(q[(s + R - m) % QR], e), el(q[(s + R + m) % QR], e));
                out[e] = point_op<R, OP>(xs[4 + e], sm, el(pv[b], e), el(kv[b], e), gxy[e] * gz, c);
            }
            float *dst = un + pc + dz;
            if (full) {
                const float4 o4 = make_float4(out[0], out[1], out[2], out[3]);
                if constexpr (PONLY) {
                    // the shell call: u_nxt is written by the call that updates every owned cell
                } else if constexpr (STREAM) {
                    st4_nt(dst, o4);
                } else {
                    st4(dst, o4);
                }
                if constexpr (PACK) {
                    // the float4 is one row of a face's R-thick layer (R = 4, nx % 4 == 0): copy it into
                    // each face slot that holds it, in the slot order of rtm_pack_halo
                    const long long nx = g.nx, ny = g.ny;
                    if (x < R) st4(po.faces + po.off[0] + ((long long)k * ny + y) * R, o4);
                    if (x >= g.nx - R) st4(po.faces + po.off[1] + ((long long)k * ny + y) * R, o4);
                    if (y < R) st4(po.faces + po.off[2] + ((long long)k * R + y) * nx + x, o4);
                    if (y >= g.ny - R) st4(po.faces + po.off[3] + ((long long)k * R + (y - (g.ny - R))) * nx + x, o4);
                    if (k < R) st4(po.faces + po.off[4] + ((long long)k * ny + y) * nx + x, o4);
                    if (k >= g.nz - R) st4(po.faces + po.off[5] + ((long long)(k - (g.nz - R)) * ny + y) * nx + x, o4);
                }
            } else if constexpr (!PONLY) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e >= elo && e < ehi) dst[e] = out[e];
            }
        }
        sk = (sk + 1 < S) ? sk + 1 : 0;
        return true;
    };
#pragma unroll 1
    for (k0_ = zs; k0_ < ze; k0_ += QR) unroll_seq(plane, std::make_integer_sequence<int, QR>{});
}

template <int R, int BX, int BY, int OP, bool PACK = false, int FL = 0>
__global__ __launch_bounds__(BX *BY) __attribute__((amdgpu_waves_per_eu(BX * BY >= 512 ? 4 : 1)))
void k_tiled(Geo g, float *un, const float *__restrict__ uc, const float *up, const float *kap, BoxList bl,
             PackOut po, const float *__restrict__ rk)
{
    __shared__ float4 lds[TileLds<R, BX, BY>::N];
    tiled_body<R, BX, BY, OP, PACK, FL>((int)blockIdx.x, lds, g, un, uc, up, kap, bl, po, rk);
}


// The shell call's x strips (radius 4: the float4 at x = 0 or x = nx - 4 of the rows y in [4, ny - 4),
// z in [4, nz - 4)) from dense face copies: one thread per row and side.  u^n at the strip and its y and
// z neighbours come from fc (u^n's face buffer), u^{n-1} from fp and kappa from fk (the same layout:
// the face slots 0 and 1 at off0 and off1), the x ghosts from gl / gr (the receive slots 0 and 1), and
// only the float4 on the inside (x = 4 or nx - 8) from the field uc.  The result goes to the face
// buffer `faces` only.  Same arithmetic, in the same order, as k_tiled.
__device__ __forceinline__ void xface_rows(long long t0, long long tstride, const Geo g,
                                           const float *__restrict__ uc, const float *__restrict__ fc,
                                           const float *__restrict__ fp, const float *__restrict__ fk,
                                           const float *__restrict__ gl, const float *__restrict__ gr,
                                           float *__restrict__ faces, long long off0, long long off1)
{
    constexpr int R = 4;
    const long long ny = g.ny, wy = g.ny - 2 * R, per = wy * (g.nz - 2 * R);
    float c[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) c[m] = g.c[m];
    for (long long t = t0; t < 2 * per; t += tstride) {
        const int side = t >= per ? 1 : 0;
        const long long r = t - side * per;
        const int y = R + (int)(r % wy), z = R + (int)(r / wy);
        const long long off = side ? off1 : off0;
        auto at = [&](int yy, int zz) { return off + ((long long)zz * ny + yy) * R; };
        const float4 xc = ld4(fc + at(y, z));
        const float4 xl = side ? ld4(uc + pidx(g, g.nx - 2 * R, y, z)) : ld4(gl + (at(y, z) - off));
        const float4 xr = side ? ld4(gr + (at(y, z) - off)) : ld4(uc + pidx(g, R, y, z));
        float4 ym[R], yp[R], zm[R], zp[R];
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            ym[m - 1] = ld4(fc + at(y - m, z));
            yp[m - 1] = ld4(fc + at(y + m, z));
            zm[m - 1] = ld4(fc + at(y, z - m));
            zp[m - 1] = ld4(fc + at(y, z + m));
        }
        const float4 pv = ld4(fp + at(y, z)), kv = ld4(fk + at(y, z));
        const int x0 = side ? g.nx - R : 0;
        const float gz = g.gz[z];
        const float xs[12] = {xl.x, xl.y, xl.z, xl.w, xc.x, xc.y, xc.z, xc.w, xr.x, xr.y, xr.z, xr.w};
        float out[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float sm[R];
#pragma unroll
            for (int m = 1; m <= R; ++m)
                sm[m - 1] = axis_sum(xs[4 + e - m], xs[4 + e + m], el(ym[m - 1], e), el(yp[m - 1], e),
                                     el(zm[m - 1], e), el(zp[m - 1], e));
            const float gxy = g.gx[x0 + e] * g.gy[y];
            out[e] = point_op<R, OP_FORWARD>(xs[4 + e], sm, el(pv, e), el(kv, e), gxy * gz, c);
        }
        st4(faces + at(y, z), make_float4(out[0], out[1], out[2], out[3]));
    }
}

// The shell call in one launch: the first xblocks workgroups walk the x-strip rows (xface_rows, a
// stride over those blocks), the rest are 32x8-thread tiles of the z slabs and y strips (faces only,
// FL has FL_PONLY).  Both parts are latency-bound and overlap in one launch (512^3: 45 us, against
// 24 + 30 us as two launches).
constexpr int kShellLds = TileLds<4, 32, 8>::N;
template <int FL>
__global__ __launch_bounds__(256) void k_shell(Geo g, const float *__restrict__ uc, const float *up, const float *kap,
                                               BoxList slabs, PackOut po, const float *__restrict__ fc,
                                               const float *__restrict__ fp, const float *__restrict__ fk,
                                               int xblocks)
{
    __shared__ float4 lds[kShellLds];
    const int b = (int)blockIdx.x;
    if (b < xblocks) {
        xface_rows((long long)b * 256 + threadIdx.x, (long long)xblocks * 256, g, uc, fc, fp, fk, po.recv[0],
                   po.recv[1], po.faces, po.off[0], po.off[1]);
    } else {
        tiled_body<4, 32, 8, OP_FORWARD, true, FL>(b - xblocks, lds, g, const_cast<float *>(uc), uc, up, kap, slabs,
                                                   po, nullptr);
    }
}

// ---------------------------------------------------------------------------------------------
// Pack / unpack of the six R-thick faces (bitwise copies), one launch each; blockIdx.y = slot.
// ---------------------------------------------------------------------------------------------
struct FaceOffsets {
    long long off[7];
};
struct FacePtrs {
    const float *p[6];
};

__device__ __forceinline__ Slab face_owned(const Geo &g, int f)
{
    const int R = g.R, nx = g.nx, ny = g.ny, nz = g.nz;
    switch (f) {
    case 0: return {0, 0, 0, R, ny, nz};
    case 1: return {nx - R, 0, 0, R, ny, nz};
    case 2: return {0, 0, 0, nx, R, nz};
    case 3: return {0, ny - R, 0, nx, R, nz};
    case 4: return {0, 0, 0, nx, ny, R};
    default: return {0, 0, nz - R, nx, ny, R};
    }
}

__device__ __forceinline__ Slab face_ghost(const Geo &g, int f)
{
    const int R = g.R, nx = g.nx, ny = g.ny, nz = g.nz;
    switch (f) {
    case 0: return {-R, 0, 0, R, ny, nz};
    case 1: return {nx, 0, 0, R, ny, nz};
    case 2: return {0, -R, 0, nx, R, nz};
    case 3: return {0, ny, 0, nx, R, nz};
    case 4: return {0, 0, -R, nx, ny, R};
    default: return {0, 0, nz, nx, ny, R};
    }
}

// The face kernels count in I: unsigned when every slot has fewer than 2^31 items (the division is
// then 32-bit, and t + stride cannot wrap), long long otherwise.
template <typename I>
__global__ __launch_bounds__(kThreads) void k_pack(Geo g, const float *__restrict__ u, float *__restrict__ faces,
                                                   FaceOffsets fo)
{
    const int f = blockIdx.y;
    const Slab s = face_owned(g, f);
    const I cnt = (I)s.wx * (I)s.wy * (I)s.wz;
    for (I t = (I)first_item(); t < cnt; t += (I)item_stride()) {
        const I row = t / (I)s.wx;
        const int i = s.ox + (int)(t - row * (I)s.wx);
        const int j = s.oy + (int)(row % (I)s.wy);
        const int k = s.oz + (int)(row / (I)s.wy);
        faces[fo.off[f] + t] = u[pidx(g, i, j, k)];
    }
}

template <typename I>
__global__ __launch_bounds__(kThreads) void k_unpack(Geo g, float *__restrict__ u, FacePtrs src)
{
    const int f = blockIdx.y;
    const Slab s = face_ghost(g, f);
    const I cnt = (I)s.wx * (I)s.wy * (I)s.wz;
    const float *p = src.p[f];
    for (I t = (I)first_item(); t < cnt; t += (I)item_stride()) {
        const I row = t / (I)s.wx;
        const int i = s.ox + (int)(t - row * (I)s.wx);
        const int j = s.oy + (int)(row % (I)s.wy);
        const int k = s.oz + (int)(row / (I)s.wy);
        u[pidx(g, i, j, k)] = p ? p[t] : 0.0f;
    }
}

// float4 forms, used when R = 4, nx % 4 == 0 and every pointer and pitch is 16-byte aligned: then each
// face row starts on a float4 boundary and one thread moves four consecutive cells.
template <typename I>
__global__ __launch_bounds__(kThreads) void k_pack4(Geo g, const float *__restrict__ u, float *__restrict__ faces,
                                                    FaceOffsets fo)
{
    const int f = blockIdx.y;
    const Slab s = face_owned(g, f);
    const I w4 = (I)(s.wx >> 2);
    const I cnt = w4 * (I)s.wy * (I)s.wz;
    for (I t = (I)first_item(); t < cnt; t += (I)item_stride()) {
        const I row = t / w4;
        const int i = s.ox + 4 * (int)(t - row * w4);
        const int j = s.oy + (int)(row % (I)s.wy);
        const int k = s.oz + (int)(row / (I)s.wy);
        st4(faces + fo.off[f] + 4 * (long long)t, ld4(u + pidx(g, i, j, k)));
    }
}

// faces[slot position of cell p] = u[p] for each owned cell p of the list in each face slot that holds
// it (a cell within R of two or three faces is in two or three slots); other indices are skipped.
__global__ __launch_bounds__(kThreads) void k_pack_cells(Geo g, const float *__restrict__ u,
                                                         const long long *__restrict__ idx, int n,
                                                         float *__restrict__ faces, FaceOffsets fo)
{
    const int R = g.R;
    const long long nx = g.nx, ny = g.ny;
    for (long long m = first_item(); m < n; m += item_stride()) {
        const long long p = idx[m];
        const long long kk = p / g.pz, rem = p - kk * g.pz;
        const long long jj = rem / g.py, ii = rem - jj * g.py;
        if (p < 0 || kk < R || kk >= (long long)g.nz + R || jj < R || jj >= (long long)g.ny + R || ii < R ||
            ii >= (long long)g.nx + R)
            continue;
        const int i = (int)ii - R, j = (int)jj - R, k = (int)kk - R;
        const float v = u[p];
        if (i < R) faces[fo.off[0] + ((long long)k * ny + j) * R + i] = v;
        if (i >= g.nx - R) faces[fo.off[1] + ((long long)k * ny + j) * R + (i - (g.nx - R))] = v;
        if (j < R) faces[fo.off[2] + ((long long)k * R + j) * nx + i] = v;
        if (j >= g.ny - R) faces[fo.off[3] + ((long long)k * R + (j - (g.ny - R))) * nx + i] = v;
        if (k < R) faces[fo.off[4] + ((long long)k * ny + j) * nx + i] = v;
        if (k >= g.nz - R) faces[fo.off[5] + ((long long)(k - (g.nz - R)) * ny + j) * nx + i] = v;
    }
}

template <typename I>
__global__ __launch_bounds__(kThreads) void k_unpack4(Geo g, float *__restrict__ u, FacePtrs src)
{
    const int f = blockIdx.y;
    const Slab s = face_ghost(g, f);
    const I w4 = (I)(s.wx >> 2);
    const I cnt = w4 * (I)s.wy * (I)s.wz;
    const float *p = src.p[f];
    for (I t = (I)first_item(); t < cnt; t += (I)item_stride()) {
        const I row = t / w4;
        const int i = s.ox + 4 * (int)(t - row * w4);
        const int j = s.oy + (int)(row % (I)s.wy);
        const int k = s.oz + (int)(row / (I)s.wy);
        st4(u + pidx(g, i, j, k), p ? ld4(p + 4 * (long long)t) : make_float4(0.f, 0.f, 0.f, 0.f));
    }
}

// The unpack for the line-aligned layout (R = 4, nx % 32 == 0, pitch_y = nx + 32, owned (0, 0, 0) on a
// 128-byte line, pitch_z a multiple of 32): the +X ghost of row j (padded x = nx+4 .. nx+7), the row's
// 24 floats of padding and the -X ghost of row j + 1 (padded x = 0 .. 3 of the next row) are exactly
// one 128-byte line, so the two x faces are written as whole lines (eight float4 per line: slot 1's
// cells, zeros in the padding, slot 0's cells) instead of two 16-byte pieces of it.  The lines that
// also hold an edge ghost (before row 0 and after row ny - 1) write only their face cells, so edges
// and corners stay untouched.  blockIdx.y = 0: the x faces (line by line); 1..4: the y and z faces
// as in k_unpack4.
template <typename I>
__global__ __launch_bounds__(kThreads) void k_unpack_lines(Geo g, float *__restrict__ u, FacePtrs src)
{
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (blockIdx.y == 0) {
        const I lines = (I)(g.ny + 1) * (I)g.nz;
        const float *s0 = src.p[0], *s1 = src.p[1];
        for (I t = (I)first_item(); t < 8 * lines; t += (I)item_stride()) {
            const I line = t >> 3;
            const int q = (int)(t & 7);
            const int jj = (int)(line % (I)(g.ny + 1));
            const int k = (int)(line / (I)(g.ny + 1));
            // the line starts at the +X ghost of row jj - 1
            float *dst = u + pidx(g, g.nx, jj - 1, k) + 4 * q;
            if (q == 0) {
                if (jj >= 1) st4(dst, s1 ? ld4(s1 + 4 * ((long long)k * g.ny + (jj - 1))) : zero4);
            } else if (q == 7) {
                if (jj < g.ny) st4(dst, s0 ? ld4(s0 + 4 * ((long long)k * g.ny + jj)) : zero4);
            } else if (jj >= 1 && jj < g.ny) {
                st4(dst, zero4);      // padding, not a cell: written only to complete the line
            }
        }
        return;
    }
    const int f = blockIdx.y + 1;
    const Slab s = face_ghost(g, f);
    const I w4 = (I)(s.wx >> 2);
    const I cnt = w4 * (I)s.wy * (I)s.wz;
    const float *p = src.p[f];
    for (I t = (I)first_item(); t < cnt; t += (I)item_stride()) {
        const I row = t / w4;
        const int i = s.ox + 4 * (int)(t - row * w4);
        const int j = s.oy + (int)(row % (I)s.wy);
        const int k = s.oz + (int)(row / (I)s.wy);
        st4(u + pidx(g, i, j, k), p ? ld4(p + 4 * (long long)t) : zero4);
    }
}

// ---------------------------------------------------------------------------------------------
// Injection, recording, imaging
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_inject(float *u, long long total, const int64_t *__restrict__ idx,
                                                     const float *__restrict__ w, const float *__restrict__ amp, int n)
{
    for (long long s = first_item(); s < n; s += item_stride()) {
        const long long p = idx[s];
        if (p >= 0 && p < total) atomicAdd(u + p, w[s] * amp[s]);
    }
}

__global__ __launch_bounds__(kThreads) void k_record(const float *__restrict__ u, long long total,
                                                     const int64_t *__restrict__ idx, float *__restrict__ out, int n)
{
    for (long long r = first_item(); r < n; r += item_stride()) {
        const long long p = idx[r];
        out[r] = (p >= 0 && p < total) ? u[p] : 0.0f;
    }
}

// k_inject then k_record in one workgroup of 1024 threads: the adds, a device-scope fence (they are
// complete and no stale line of u is read), a barrier, then the gathers, so a receiver on a source cell
// records the injected value.  For short lists, where each launch is mostly its own start-up.
constexpr int kInjectRecordThreads = 1024;
__global__ __launch_bounds__(kInjectRecordThreads) void k_inject_record(float *u, long long total, const int64_t *__restrict__ sidx,
                                                            const float *__restrict__ w, const float *__restrict__ amp,
                                                            int ns, const int64_t *__restrict__ ridx,
                                                            float *__restrict__ out, int nr)
{
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        const long long p = sidx[s];
        if (p >= 0 && p < total) atomicAdd(u + p, w[s] * amp[s]);
    }
    __threadfence();
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        const long long p = ridx[r];
        out[r] = (p >= 0 && p < total) ? u[p] : 0.0f;
    }
}

// Owned-cell elementwise kernels walk the owned rows (j, k): one wave per row (a grid-stride loop over
// rows with 64-bit counters), its lanes over x, four cells per lane when VEC (every row's owned cells
// then start on a 16-byte boundary: R % 4 == 0, nx % 4 == 0 and both pitches multiples of 4).  One
// division per row instead of three 64-bit divisions per cell keeps these kernels on HBM rather than
// on integer arithmetic.  f(p, c, k) handles the cell(s) at padded index p and compact index c
// ((k ny + j) nx + i) in plane k.
constexpr int kRowWaves = kThreads / 64;

template <bool VEC, typename F>
__device__ __forceinline__ void owned_rows(const Geo &g, F &&f)
{
    const int lane = threadIdx.x & 63;
    const long long rows = (long long)g.ny * g.nz;
    const long long wstride = (long long)gridDim.x * kRowWaves;
    for (long long r = (long long)blockIdx.x * kRowWaves + (threadIdx.x >> 6); r < rows; r += wstride) {
        const int k = (int)(r / g.ny), j = (int)(r - (long long)k * g.ny);
        const long long p0 = pidx(g, 0, j, k), c0 = r * g.nx;
        if constexpr (VEC) {
            for (int i = 4 * lane; i < g.nx; i += 256) f(p0 + i, c0 + i, k);
        } else {
            for (int i = lane; i < g.nx; i += 64) f(p0 + i, c0 + i, k);
        }
    }
}

template <bool VEC, bool NT = false>
__global__ __launch_bounds__(kThreads) void k_image(Geo g, float *image, const float *__restrict__ src,
                                                    const float *__restrict__ rcv, float weight)
{
    owned_rows<VEC>(g, [&](long long p, long long, int) {
        if constexpr (VEC) {
            const float4 s4 = NT ? ld4_nt(src + p) : ld4(src + p), r4 = NT ? ld4_nt(rcv + p) : ld4(rcv + p);
            float4 o = NT ? ld4_nt(image + p) : ld4(image + p);
            o.x = __builtin_fmaf(weight * s4.x, r4.x, o.x);
            o.y = __builtin_fmaf(weight * s4.y, r4.y, o.y);
            o.z = __builtin_fmaf(weight * s4.z, r4.z, o.z);
            o.w = __builtin_fmaf(weight * s4.w, r4.w, o.w);
            if constexpr (NT)
                st4_nt(image + p, o);
            else
                st4(image + p, o);
        } else {
            image[p] = __builtin_fmaf(weight * src[p], rcv[p], image[p]);
        }
    });
}

template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_kappa(Geo g, float *__restrict__ kappa, const float *__restrict__ v,
                                                    float s)
{
    owned_rows<VEC>(g, [&](long long p, long long c, int) {
        if constexpr (VEC) {
            const float4 v4 = ld4(v + c);
            const float a0 = v4.x * s, a1 = v4.y * s, a2 = v4.z * s, a3 = v4.w * s;
            st4(kappa + p, make_float4(a0 * a0, a1 * a1, a2 * a2, a3 * a3));
        } else {
            const float a = v[c] * s;
            kappa[p] = a * a;
        }
    });
}

// count += the number of owned cells of u that are not finite (NaN or infinite: all exponent bits
// set), one atomic add per wave.
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_count_nonfinite(Geo g, const float *__restrict__ u,
                                                              unsigned *__restrict__ count)
{
    auto bad = [](float x) -> unsigned { return ((__float_as_uint(x) >> 23) & 0xFFu) == 0xFFu ? 1u : 0u; };
    unsigned n = 0;
    owned_rows<VEC>(g, [&](long long p, long long, int) {
        if constexpr (VEC) {
            const float4 v = ld4(u + p);
            n += bad(v.x) + bad(v.y) + bad(v.z) + bad(v.w);
        } else {
            n += bad(u[p]);
        }
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, n);
}

// ---------------------------------------------------------------------------------------------
// Adjoint-state gradient helpers
// ---------------------------------------------------------------------------------------------
// w = kappa g mu on owned cells (the field the adjoint stencil differentiates).
__global__ __launch_bounds__(kThreads) void k_adjoint_weight(Geo g, float *__restrict__ w, const float *__restrict__ mu,
                                                             const float *__restrict__ kap)
{
    const long long nxy = (long long)g.nx * g.ny;
    for (long long t = first_item(); t < nxy * g.nz; t += item_stride()) {
        const int i = (int)(t % g.nx);
        const int j = (int)((t / g.nx) % g.ny);
        const int k = (int)(t / nxy);
        const long long p = pidx(g, i, j, k);
        w[p] = (kap[p] * sponge(g, i, j, k)) * mu[p];
    }
}

// resid = d - obs and misfit += 1/2 sum resid^2, summed in FP64 by one workgroup: each thread adds a
// fixed strided subset in order and the partial sums meet in a fixed tree, so the result does not
// depend on scheduling (bitwise reproducible).
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_residual(const float *__restrict__ d, const float *__restrict__ obs,
                                                             float *__restrict__ resid, long long n, double *misfit)
{
    double acc = 0.0;
    for (long long t = threadIdx.x; t < n; t += kReduceThreads) {
        const float r = d[t] - obs[t];
        resid[t] = r;
        acc += (double)r * (double)r;
    }
    __shared__ double red[kReduceThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *misfit += 0.5 * red[0];
}

// The same over `nb` contiguous chunks of the samples, one workgroup each: chunk b is
// [b * chunk, min(n, (b + 1) * chunk)), its threads stride through it in order and meet in a fixed
// tree, and the chunk's FP64 sum of squares goes to part[b]; k_residual_final adds part[0..nb) in
// order.  The order depends only on n and nb, so the result is the same on every call.
constexpr int kChunkThreads = 256;
__global__ __launch_bounds__(kChunkThreads) void k_residual_chunks(const float *__restrict__ d,
                                                                   const float *__restrict__ obs,
                                                                   float *__restrict__ resid, long long n,
                                                                   long long chunk, double *__restrict__ part)
{
    const long long lo = (long long)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double acc = 0.0;
    for (long long t = lo + threadIdx.x; t < hi; t += kChunkThreads) {
        const float r = d[t] - obs[t];
        resid[t] = r;
        acc += (double)r * (double)r;
    }
    __shared__ double red[kChunkThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kChunkThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kReduceThreads) void k_residual_final(const double *__restrict__ part, int nb,
                                                                   double *misfit)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kReduceThreads) acc += part[b];
    __shared__ double red[kReduceThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *misfit += 0.5 * red[0];
}

// grad_v (compact, x fastest) = 2 v (dt/h)^2 grad_kappa (the chain rule through kappa = (v dt/h)^2).
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_velocity_gradient(Geo g, float *__restrict__ gv,
                                                                const float *__restrict__ gk,
                                                                const float *__restrict__ v, float s2)
{
    const float two_s2 = 2.0f * s2;
    owned_rows<VEC>(g, [&](long long p, long long c, int) {
        if constexpr (VEC) {
            const float4 v4 = ld4(v + c), k4 = ld4(gk + p);
            st4(gv + c, make_float4(two_s2 * v4.x * k4.x, two_s2 * v4.y * k4.y, two_s2 * v4.z * k4.z,
                                    two_s2 * v4.w * k4.w));
        } else {
            gv[c] = two_s2 * v[c] * gk[p];
        }
    });
}

// kg[r] = kappa g and inv_kg[r] = 1 / (kappa g) at the owned cell of padded index idx[r] (the factor
// kappa (gxy gz) in the order the adjoint kernel forms kappa g mu); 0 for an index that is not an owned
// cell.  Either output may be NULL.
__global__ __launch_bounds__(kThreads) void k_scaled_factors(Geo g, const float *__restrict__ kap,
                                                             const long long *__restrict__ idx, int n,
                                                             float *__restrict__ kg, float *__restrict__ inv_kg)
{
    const int R = g.R;
    for (long long r = first_item(); r < n; r += item_stride()) {
        const long long p = idx[r];
        const long long kk = p / g.pz, rem = p - kk * g.pz;
        const long long jj = rem / g.py, ii = rem - jj * g.py;
        float f = 0.0f, fi = 0.0f;
        if (p >= 0 && kk >= R && kk < (long long)g.nz + R && jj >= R && jj < (long long)g.ny + R && ii >= R &&
            ii < (long long)g.nx + R) {
            const int i = (int)ii - R, j = (int)jj - R, k = (int)kk - R;
            f = kap[p] * ((g.gx[i] * g.gy[j]) * g.gz[k]);
            fi = 1.0f / f;
        }
        if (kg) kg[r] = f;
        if (inv_kg) inv_kg[r] = fi;
    }
}

__global__ __launch_bounds__(kThreads) void k_record_weighted(const float *__restrict__ u, long long total,
                                                              const int64_t *__restrict__ idx,
                                                              const float *__restrict__ w, float *__restrict__ out,
                                                              int n)
{
    for (long long r = first_item(); r < n; r += item_stride()) {
        const long long p = idx[r];
        out[r] = (p >= 0 && p < total) ? w[r] * u[p] : 0.0f;
    }
}

// grad_v (compact) = 2 G / v: the chain rule for the gradient accumulated from the scaled adjoint state
// w = kappa g mu (G = sum w L u = kappa dJ/dkappa, and dkappa/dv = 2 kappa / v).
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_velocity_gradient_scaled(Geo g, float *__restrict__ gv,
                                                                       const float *__restrict__ G,
                                                                       const float *__restrict__ v)
{
    owned_rows<VEC>(g, [&](long long p, long long c, int) {
        if constexpr (VEC) {
            const float4 v4 = ld4(v + c), k4 = ld4(G + p);
            st4(gv + c, make_float4((2.0f * k4.x) / v4.x, (2.0f * k4.y) / v4.y, (2.0f * k4.z) / v4.z,
                                    (2.0f * k4.w) / v4.w));
        } else {
            gv[c] = (2.0f * G[p]) / v[c];
        }
    });
}

// ---------------------------------------------------------------------------------------------
// Reduced-precision snapshots: one FP32 scale per z plane (slab) and 16-bit codes
// ---------------------------------------------------------------------------------------------
// FP32 -> BF16 with round-to-nearest-even on the bit pattern (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t c) { return __uint_as_float((uint32_t)c << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float x)
{
    const _Float16 h = (_Float16)x;    // hardware conversion, round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t c) { return (float)__builtin_bit_cast(_Float16, c); }

// scales[k] = max |u| over the owned cells of plane k (one workgroup per plane).
// scales[k] = max |u| over owned plane k: one 1024-thread workgroup per plane with four loads in
// flight per thread (float4 rows when VEC: nx % 4 == 0 and every row start 16-byte aligned), then a
// wave-shuffle and LDS reduction.  A maximum is exact in any order.
constexpr int kAbsmaxThreads = 1024;

template <bool VEC>
__global__ __launch_bounds__(kAbsmaxThreads) void k_plane_absmax(Geo g, const float *__restrict__ u,
                                                                 float *__restrict__ scales)
{
    const int k = blockIdx.x;
    float m = 0.0f;
    if constexpr (VEC) {
        const long long w4 = g.nx >> 2;
        const long long n4 = w4 * g.ny;
        for (long long t0 = threadIdx.x; t0 < n4; t0 += 4 * kAbsmaxThreads) {
            float4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long long t = t0 + q * kAbsmaxThreads;
                v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < n4) {
                    const int j = (int)(t / w4), i4 = (int)(t - j * w4);
                    v[q] = ld4(u + pidx(g, 4 * i4, j, k));
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                m = fmaxf(m, fmaxf(fmaxf(fabsf(v[q].x), fabsf(v[q].y)), fmaxf(fabsf(v[q].z), fabsf(v[q].w))));
        }
    } else {
        const long long nxy = (long long)g.nx * g.ny;
        for (long long t0 = threadIdx.x; t0 < nxy; t0 += 4 * kAbsmaxThreads) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long long t = t0 + q * kAbsmaxThreads;
                v[q] = 0.0f;
                if (t < nxy) {
                    const int j = (int)(t / g.nx), i = (int)(t - (long long)j * g.nx);
                    v[q] = u[pidx(g, i, j, k)];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) m = fmaxf(m, fabsf(v[q]));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    __shared__ float red[kAbsmaxThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x < 64) {
        m = threadIdx.x < kAbsmaxThreads / 64 ? red[threadIdx.x] : 0.0f;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if (threadIdx.x == 0) scales[k] = m;
    }
}

// codes[(k ny + j) nx + i] = RNE(u / scales[k]) in the 16-bit format; a zero scale gives zero codes.
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_encode(Geo g, const float *__restrict__ u, const float *__restrict__ scales,
                                                     uint16_t *__restrict__ codes, int fmt)
{
    auto code = [&](float x, float sc) -> uint32_t {
        const float q = sc > 0.0f ? x / sc : 0.0f;
        return fmt == RTM_SNAP_BF16 ? f32_to_bf16_rne(q) : f32_to_f16_rne(q);
    };
    owned_rows<VEC>(g, [&](long long p, long long c, int k) {
        const float sc = scales[k];
        if constexpr (VEC) {
            const float4 u4 = ld4(u + p);
            uint2 w;
            w.x = code(u4.x, sc) | (code(u4.y, sc) << 16);
            w.y = code(u4.z, sc) | (code(u4.w, sc) << 16);
            *reinterpret_cast<uint2 *>(codes + c) = w;
        } else {
            codes[c] = (uint16_t)code(u[p], sc);
        }
    });
}

// image += weight * (decode(code) * scale) * rcv on owned cells.
template <bool VEC, bool NT = false>
__global__ __launch_bounds__(kThreads) void k_image_coded(Geo g, float *image, const uint16_t *__restrict__ codes,
                                                          const float *__restrict__ scales, int fmt,
                                                          const float *__restrict__ rcv, float weight)
{
    auto value = [&](uint32_t c, float sc) {
        return (fmt == RTM_SNAP_BF16 ? bf16_to_f32((uint16_t)c) : f16_to_f32((uint16_t)c)) * sc;
    };
    owned_rows<VEC>(g, [&](long long p, long long c, int k) {
        const float sc = scales[k];
        if constexpr (VEC) {
            typedef unsigned u2v __attribute__((ext_vector_type(2)));
            uint2 w;
            if constexpr (NT) {
                const u2v t = __builtin_nontemporal_load(reinterpret_cast<const u2v *>(codes + c));
                w = make_uint2(t.x, t.y);
            } else {
                w = *reinterpret_cast<const uint2 *>(codes + c);
            }
            const float4 r4 = NT ? ld4_nt(rcv + p) : ld4(rcv + p);
            float4 o = NT ? ld4_nt(image + p) : ld4(image + p);
            o.x = __builtin_fmaf(weight * value(w.x & 0xFFFFu, sc), r4.x, o.x);
            o.y = __builtin_fmaf(weight * value(w.x >> 16, sc), r4.y, o.y);
            o.z = __builtin_fmaf(weight * value(w.y & 0xFFFFu, sc), r4.z, o.z);
            o.w = __builtin_fmaf(weight * value(w.y >> 16, sc), r4.w, o.w);
            if constexpr (NT)
                st4_nt(image + p, o);
            else
                st4(image + p, o);
        } else {
            image[p] = __builtin_fmaf(weight * value(codes[c], sc), rcv[p], image[p]);
        }
    });
}

// ---------------------------------------------------------------------------------------------
// Host side: validation, device check, launch configuration
// ---------------------------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::atomic<int> g_dev_ok[kMaxDevices];   // 0 unknown, 1 gfx950, -1 other

struct Options {
    std::atomic<int> interior_variant{2};  // 0: 16x16 threads (64 x 16 cells), 1: 32x8, 2: 16x8, 3: scalar,
                                           // 4: 32x16 (128 x 16 cells, two workgroups per CU), 5: 16x32
    std::atomic<int> whole_variant{6};     // tile shape of the one-launch whole step (not 3); 6 = by radius
    std::atomic<int> zchunk{0};            // 0: automatic
    std::atomic<int> xcd_remap{1};
    std::atomic<int> halo_x_width{64};     // x strips of the halo region
    std::atomic<int> halo_z_width{0};      // z slabs of the halo region (0: R planes)
    std::atomic<int> halo_y_width{8};      // y strips of the halo region (8 rows: the 512^3 interior box
                                           // is 62 rows of 16x8 tiles, 744 workgroups in 2 chunks on 256
                                           // CUs; 16 rows gave 720, and a 1% slower step)
    std::atomic<int> halo_variant{0};      // tile shape of the halo call (as interior_variant; 5: 16x32)
    std::atomic<int> unpack_lines{1};      // 1: x-face ghosts unpacked as whole lines where the layout allows
    std::atomic<int> tile_flags{FL_NT};    // FL_NT (streaming hints, default) | FL_XSHUF (lane shifts)
    std::atomic<int> markers{0};           // roctx ranges around the per-step calls
};
Options g_opt;

// Phase markers (RTM_OPT_MARKERS): a roctx range named after the call around each per-step call, so
// a trace (rocprofv3 --marker-trace) shows every step's phase sequence on the host timeline.  The
// roctx library is opened when the option is first set; nothing links against it.
struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};

const Roctx &roctx()
{
    static const Roctx api = [] {
        Roctx r;
        void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
        if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_GLOBAL);
        if (h) {
            r.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
            r.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
            if (!r.push || !r.pop) r.push = nullptr, r.pop = nullptr;
        }
        return r;
    }();
    return api;
}

struct Marker {
    bool on;
    explicit Marker(const char *name) : on(g_opt.markers.load(std::memory_order_relaxed) != 0)
    {
        if (on) roctx().push(name);
    }
    ~Marker()
    {
        if (on) roctx().pop();
    }
    Marker(const Marker &) = delete;
    Marker &operator=(const Marker &) = delete;
};

int check_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RTM_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return RTM_EDEVICE;
    int st = g_dev_ok[dev].load(std::memory_order_relaxed);
    if (st == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RTM_EDEVICE;
        st = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
        g_dev_ok[dev].store(st, std::memory_order_relaxed);
    }
    return st == 1 ? RTM_OK : RTM_EDEVICE;
}

int check_grid(const rtm_grid *gr)
{
    if (!gr) return RTM_EINVAL;
    const int R = gr->radius;
    if (R != 2 && R != 4) return RTM_EINVAL;
    if (gr->nx < 2 * R || gr->ny < 2 * R || gr->nz < 2 * R) return RTM_EINVAL;
    if (gr->pitch_y < (int64_t)gr->nx + 2 * R) return RTM_EINVAL;
    if (gr->pitch_z < gr->pitch_y * ((int64_t)gr->ny + 2 * R)) return RTM_EINVAL;
    if (!gr->gx || !gr->gy || !gr->gz) return RTM_EINVAL;
    return RTM_OK;
}

Geo make_geo(const rtm_grid *gr)
{
    Geo g;
    g.nx = gr->nx;
    g.ny = gr->ny;
    g.nz = gr->nz;
    g.R = gr->radius;
    g.py = gr->pitch_y;
    g.pz = gr->pitch_z;
    for (int m = 0; m < 5; ++m) g.c[m] = (m <= gr->radius) ? gr->c[m] : 0.0f;
    g.gx = gr->gx;
    g.gy = gr->gy;
    g.gz = gr->gz;
    return g;
}

long long padded_total(const rtm_grid *gr) { return gr->pitch_z * ((long long)gr->nz + 2 * gr->radius); }

int launch_status()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTM_OK : RTM_ELAUNCH;
}

// Workgroups for n items of an elementwise kernel (which strides by the grid beyond the cap).
constexpr long long kMaxBlocks = 1ll << 20;
// rtm_inject_record: at most this many sources plus receivers go to one workgroup
constexpr long long kInjectRecordOneGroup = 4096;
unsigned blocks_for(long long n) { return (unsigned)std::min((n + kThreads - 1) / kThreads, kMaxBlocks); }

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Workgroups for the owned-row kernels (kRowWaves rows each, grid-stride beyond the cap), and whether
// every row's owned cells start on a float4 boundary of the padded layout.
unsigned row_blocks(const Geo &g)
{
    const long long rows = (long long)g.ny * g.nz;
    return (unsigned)std::min((rows + kRowWaves - 1) / kRowWaves, kMaxBlocks);
}
bool rows_vec(const Geo &g) { return g.R % 4 == 0 && g.nx % 4 == 0 && g.py % 4 == 0 && g.pz % 4 == 0; }

int cu_count()
{
    static std::atomic<int> cached{0};
    int n = cached.load(std::memory_order_relaxed);
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cached.store(n, std::memory_order_relaxed);
    }
    return n;
}

// z chunk of a launch over one deep box of `tiles` XY tiles and depth wz, for workgroups of
// `waves` wavefronts.  Each chunk re-reads 2R planes it does not write, and the launch lasts about as
// long as its busiest CU, which holds k = ceil(tiles * nzc / CUs) workgroups.  A CU streams at full
// rate only once it holds about 6 wavefronts (one 32x8 workgroup, 4 waves, runs at about 3/4 of it),
// so the cost counts at least 6 / waves workgroups per CU:
//     cost(nzc) = max(k, 6 / waves) * (wz / nzc + 2R)    (in tile-planes).
// Among chunkings within 3% of the least cost the one with the fewest workgroups wins: fewer,
// longer streams use HBM better.  At 512^3 this gives 2 chunks for the interior call (720
// workgroups of 16x8: 269-276 us; 1 chunk 313 us, 3 chunks 301 us), for every tile shape of the
// one-launch call (32x8 threads: 343 us against 462 us for 1 chunk; 32x16: 376 us, 1 chunk 597 us,
// 3 chunks 427 us) and for the direct adjoint step (500 against 643 us for 1 chunk).
int balanced_zchunk(int tiles, int wz, int R, int cus, int waves)
{
    const double min_k = 6.0 / std::max(1, waves);
    const int max_nzc = std::max(1, wz / 16);
    double best = -1;
    double cost[64 + 1];
    const int n_try = std::min(max_nzc, 64);
    for (int nzc = 1; nzc <= n_try; ++nzc) {
        const int zc = (wz + nzc - 1) / nzc;
        const long long blocks = (long long)tiles * ((wz + zc - 1) / zc);
        const double k = (double)((blocks + cus - 1) / cus);
        cost[nzc] = std::max(k, min_k) * (double)(zc + 2 * R);
        if (best < 0 || cost[nzc] < best) best = cost[nzc];
    }
    for (int nzc = 1; nzc <= n_try; ++nzc)   // fewest workgroups first
        if (cost[nzc] <= best * 1.03) return (wz + nzc - 1) / nzc;
    return wz;
}

// The box list of a tiled launch over up to kMaxBoxes boxes {x0, x1, y0, y1, z0, z1} (empty ones
// skipped), its z chunking and workgroup order; zc_hint > 0: the z chunk when RTM_OPT_ZCHUNK is
// automatic.  RTM_EINVAL when the launch would need 2^31 workgroups or more.
template <int R, int BX, int BY>
int make_boxlist(const Geo &g, const int (*boxes)[6], int nbox, int remap, int zc_hint, BoxList &bl)
{
    constexpr int TX = 4 * BX;
    std::memset(&bl, 0, sizeof(bl));
    int tiles = 0, wz = 0;
    for (int i = 0; i < nbox; ++i) {
        const int *b = boxes[i];
        if (b[1] <= b[0] || b[3] <= b[2] || b[5] <= b[4]) continue;
        Box &x = bl.b[bl.nbox++];
        x.x0 = b[0];
        x.x1 = b[1];
        x.y0 = b[2];
        x.y1 = b[3];
        x.z0 = b[4];
        x.z1 = b[5];
        x.X0 = x.x0 - ((x.x0 + R) & 3);
        x.ntx = (x.x1 - x.X0 + TX - 1) / TX;
        x.nty = (x.y1 - x.y0 + BY - 1) / BY;
        if (x.z1 - x.z0 > 2 * R) {           // deep boxes share the z chunking; thin slabs are one chunk
            tiles += x.ntx * x.nty;
            wz = std::max(wz, x.z1 - x.z0);
        }
    }
    if (bl.nbox == 0) return RTM_OK;
    (void)g;
    int zc = g_opt.zchunk.load(std::memory_order_relaxed);
    if (zc <= 0 && zc_hint > 0) {
        zc = zc_hint;
    } else if (zc <= 0 && tiles > 0 && R <= 2) {
        // Narrow stencils: short chunks.  A chunk re-reads 2R planes it does not write, only 25% at
        // 16 planes for R = 2, and several short waves of workgroups balance better than one long
        // one (384^3 whole step: 237 us at 16 planes against 266 us for one wave).
        zc = 16;
    } else if (zc <= 0 && tiles > 0 && bl.nbox == 1) {
        zc = balanced_zchunk(tiles, wz, R, cu_count(), (BX * BY + 63) / 64);
    } else if (zc <= 0 && tiles > 0) {
        // The halo call's mix of thin slabs and deep strips: short chunks of 12 planes for its deep
        // strips, many small workgroups that fill the chip evenly (512^3 halo call with the pack:
        // 155 us, against 174 us with one wave of resident workgroups, about 51-plane chunks;
        // 8 planes 160, 16 planes 157, 24 planes 167 us).
        zc = 12;
    }
    if (zc <= 0) zc = 1 << 30;
    long long nb = 0;
    for (int i = 0; i < bl.nbox; ++i) {
        Box &x = bl.b[i];
        x.zchunk = std::min(zc, x.z1 - x.z0);
        x.nzc = (x.z1 - x.z0 + x.zchunk - 1) / x.zchunk;
        x.nblk = x.ntx * x.nty * x.nzc;
        nb += x.nblk;
    }
    if (nb >= (1ll << 31)) return RTM_EINVAL;
    bl.nblk = (int)nb;
    bl.remap = remap >= 0 ? remap : g_opt.xcd_remap.load(std::memory_order_relaxed);
    return RTM_OK;
}

// Launch the tiled kernel over up to kMaxBoxes boxes (make_boxlist).
// rk: kappa for OP_ADJOINT (see k_tiled), unused otherwise.
template <int R, int BX, int BY, int OP, bool PACK = false, int FL = 0>
int launch_tiled(const Geo &g, float *un, const float *uc, const float *up, const float *kap, const int (*boxes)[6],
                 int nbox, hipStream_t st, const PackOut *po = nullptr, const float *rk = nullptr, int remap = -1,
                 int zc_hint = 0)
{
    BoxList bl;
    const int rc = make_boxlist<R, BX, BY>(g, boxes, nbox, remap, zc_hint, bl);
    if (rc != RTM_OK || bl.nblk == 0) return rc;
    PackOut pk;
    std::memset(&pk, 0, sizeof(pk));
    if (po) pk = *po;
    hipLaunchKernelGGL((k_tiled<R, BX, BY, OP, PACK, FL>), dim3((unsigned)bl.nblk), dim3(BX * BY), 0, st, g, un, uc, up,
                       kap, bl, pk, rk);
    return launch_status();
}

template <int R, int OP, bool PACK = false, int FL = 0>
int launch_tiled_flags(int var, const Geo &g, float *un, const float *uc, const float *up, const float *kap,
                       const int (*boxes)[6], int nbox, hipStream_t st, const PackOut *po, const float *rk,
                       int remap)
{
    switch (var) {
    case 1: return launch_tiled<R, 32, 8, OP, PACK, FL>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 2: return launch_tiled<R, 16, 8, OP, PACK, FL>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 4: return launch_tiled<R, 32, 16, OP, PACK, FL>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 5: return launch_tiled<R, 16, 32, OP, PACK, FL>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    default: return launch_tiled<R, 16, 16, OP, PACK, FL>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    }
}

template <int R, int OP, bool PACK = false>
int launch_tiled_variant(int var, const Geo &g, float *un, const float *uc, const float *up, const float *kap,
                         const int (*boxes)[6], int nbox, hipStream_t st, const PackOut *po = nullptr,
                         const float *rk = nullptr, bool slots = false, int remap = -1)
{
    // kernel flags: streaming hints for every operation; lane shifts for the radius-4 forward update;
    // ghosts from the receive slots for the radius-4 halo call that packs
    const int fl = g_opt.tile_flags.load(std::memory_order_relaxed);
    if constexpr (R == 4 && OP == OP_FORWARD && PACK) {
        if (slots) {
            if (fl & FL_NT)
                return launch_tiled_flags<R, OP, PACK, FL_NT | FL_SLOTS>(var, g, un, uc, up, kap, boxes, nbox, st, po,
                                                                         rk, remap);
            return launch_tiled_flags<R, OP, PACK, FL_SLOTS>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
        }
    }
    if constexpr (R == 4 && OP == OP_FORWARD && !PACK) {
        if (slots) {
            if (fl & FL_NT)
                return launch_tiled_flags<R, OP, PACK, FL_NT | FL_SLOTS>(var, g, un, uc, up, kap, boxes, nbox, st, po,
                                                                         rk, remap);
            return launch_tiled_flags<R, OP, PACK, FL_SLOTS>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
        }
    }
    if (slots) return RTM_EINVAL;
    if constexpr (R == 4 && OP == OP_FORWARD && !PACK) {
        switch (fl) {
        case FL_NT: return launch_tiled_flags<R, OP, PACK, FL_NT>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
        case FL_XSHUF:
            return launch_tiled_flags<R, OP, PACK, FL_XSHUF>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
        case FL_NT | FL_XSHUF:
            return launch_tiled_flags<R, OP, PACK, FL_NT | FL_XSHUF>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
        default: break;
        }
    } else {
        if (fl & FL_NT) return launch_tiled_flags<R, OP, PACK, FL_NT>(var, g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    }
    switch (var) {
    case 1: return launch_tiled<R, 32, 8, OP, PACK>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 2: return launch_tiled<R, 16, 8, OP, PACK>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 4: return launch_tiled<R, 32, 16, OP, PACK>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    case 5: return launch_tiled<R, 16, 32, OP, PACK>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    default: return launch_tiled<R, 16, 16, OP, PACK>(g, un, uc, up, kap, boxes, nbox, st, po, rk, remap);
    }
}

// The halo region: the two R-thick z slabs, the two hy-row y strips between them and the two wx-wide
// x strips between those.  The widths depend only on the grid and the options (never on pointers),
// so callers can tell which call updates a given cell (rtm_halo_region).
struct Region {
    int wx, hy, hz, R;
};

Region halo_region(int nx, int ny, int nz, int R)
{
    Region r;
    r.R = R;
    r.wx = std::max(R, std::min(g_opt.halo_x_width.load(std::memory_order_relaxed), nx / 2));
    r.hy = std::max(R, std::min(g_opt.halo_y_width.load(std::memory_order_relaxed), ny / 2));
    const int hz = g_opt.halo_z_width.load(std::memory_order_relaxed);
    r.hz = hz > 0 ? std::max(R, std::min(hz, nz / 2)) : R;
    return r;
}

int halo_boxes(const Geo &g, const Region &r, int boxes[6][6])
{
    const int nx = g.nx, ny = g.ny, nz = g.nz, hz = r.hz;
    const int b[6][6] = {
        {0, nx, 0, ny, 0, hz},                         // -Z slab
        {0, nx, 0, ny, nz - hz, nz},                   // +Z slab
        {0, nx, 0, r.hy, hz, nz - hz},                 // -Y strip
        {0, nx, ny - r.hy, ny, hz, nz - hz},           // +Y strip
        {0, r.wx, r.hy, ny - r.hy, hz, nz - hz},       // -X strip
        {nx - r.wx, nx, r.hy, ny - r.hy, hz, nz - hz}, // +X strip
    };
    std::memcpy(boxes, b, sizeof(b));
    return 6;
}

bool vector_path(const Geo &g, const float *un, const float *uc, const float *up, const float *kap)
{
    return g_opt.interior_variant.load(std::memory_order_relaxed) != 3 && aligned16(un) && aligned16(uc) &&
           aligned16(up) && aligned16(kap) && (g.py % 4 == 0) && (g.pz % 4 == 0);
}

template <int R, int OP>
int launch_box_scalar(const Geo &g, float *un, const float *uc, const float *up, const float *kap, const int *b,
                      hipStream_t st)
{
    const long long n = (long long)std::max(0, b[1] - b[0]) * std::max(0, b[3] - b[2]) * std::max(0, b[5] - b[4]);
    if (n <= 0) return RTM_OK;
    hipLaunchKernelGGL((k_box<R, OP>), dim3(blocks_for(n)), dim3(kThreads), 0, st, g, un, uc, up, kap, b[0], b[1], b[2],
                       b[3], b[4], b[5]);
    return launch_status();
}

template <int R, int OP = OP_FORWARD>
int launch_halo(const Geo &g, float *un, const float *uc, const float *up, const float *kap, hipStream_t st)
{
    const Region r = halo_region(g.nx, g.ny, g.nz, R);
    int boxes[6][6];
    const int nb = halo_boxes(g, r, boxes);
    if (vector_path(g, un, uc, up, kap))
        return launch_tiled_variant<R, OP>(g_opt.halo_variant.load(std::memory_order_relaxed), g, un, uc, up, kap,
                                           boxes, nb, st);
    for (int i = 0; i < nb; ++i) {
        const int rc = launch_box_scalar<R, OP>(g, un, uc, up, kap, boxes[i], st);
        if (rc != RTM_OK) return rc;
    }
    return RTM_OK;
}

// The halo call that also writes the six faces (radius 4, float4 layout; see rtm_step_halo_pack);
// with `slots`, it reads the ghosts of u_cur from po.recv (rtm_step_halo_pack_slots).
int launch_halo_pack(const Geo &g, float *un, const float *uc, const float *up, const float *kap, const PackOut &po,
                     hipStream_t st, bool slots = false)
{
    const Region r = halo_region(g.nx, g.ny, g.nz, 4);
    int boxes[6][6];
    const int nb = halo_boxes(g, r, boxes);
    return launch_tiled_variant<4, OP_FORWARD, true>(g_opt.halo_variant.load(std::memory_order_relaxed), g, un, uc,
                                                     up, kap, boxes, nb, st, &po, nullptr, slots);
}

// The shell call (radius 4, ghosts from po.recv): the owned cells within R of a face, written to the
// face buffer only.  With dense face copies of u_cur, u_prv and kappa (fc, fp, fk): one launch of
// k_shell, the two 4-column x strips as one thread per row (xface_rows, one float4 per row read from
// the field) and the two z slabs and the two y strips between them as 32x8-thread tiles in 16-plane
// z chunks (44-49 us at 512^3).  Without them, or on grids too small for the row walk: the slabs and
// strips in one launch of those tiles, then the x strips in 2x32-thread tiles (8 columns: the centre
// float4 and its inside neighbour) in 32-plane chunks, which read three float4s of separate lines per
// row and plane from the fields (68-70 us at 512^3).
int launch_shell_pack(const Geo &g, const float *uc, const float *up, const float *kap, const float *fc,
                      const float *fp, const float *fk, const PackOut &po, hipStream_t st)
{
    constexpr int R = 4;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int zl = std::min(R, nz), zh = std::max(R, nz - R), yl = std::min(R, ny), yh = std::max(R, ny - R);
    const int slabs[4][6] = {
        {0, nx, 0, ny, 0, zl},                 // -Z slab
        {0, nx, 0, ny, zh, nz},                // +Z slab
        {0, nx, 0, yl, R, nz - R},             // -Y strip
        {0, nx, yh, ny, R, nz - R},            // +Y strip
    };
    const int cols[2][6] = {
        {0, std::min(R, nx), R, ny - R, R, nz - R},          // -X strip
        {std::max(R, nx - R), nx, R, ny - R, R, nz - R},     // +X strip
    };
    // u_nxt is never written (FL_PONLY); the tile code forms its addresses from uc
    float *un = const_cast<float *>(uc);
    const bool nt = (g_opt.tile_flags.load(std::memory_order_relaxed) & FL_NT) != 0;
    constexpr int F1 = FL_NT | FL_SLOTS | FL_PONLY, F0 = FL_SLOTS | FL_PONLY;
    if (fc && nx >= 2 * R && ny > 2 * R && nz > 2 * R) {
        BoxList bs;
        const int rc = make_boxlist<R, 32, 8>(g, slabs, 4, -1, 16, bs);
        if (rc != RTM_OK) return rc;
        const long long rows = 2ll * (ny - 2 * R) * (nz - 2 * R);
        const int xblocks = (int)((rows + 255) / 256);      // one row per thread (45 us at 512^3)
        const long long nb = (long long)xblocks + bs.nblk;
        if (nb >= (1ll << 31)) return RTM_EINVAL;
        if (nt)
            hipLaunchKernelGGL((k_shell<F1>), dim3((unsigned)nb), dim3(256), 0, st, g, uc, up, kap, bs, po, fc, fp, fk,
                               xblocks);
        else
            hipLaunchKernelGGL((k_shell<F0>), dim3((unsigned)nb), dim3(256), 0, st, g, uc, up, kap, bs, po, fc, fp, fk,
                               xblocks);
        return launch_status();
    }
    int rc = nt ? launch_tiled<R, 32, 8, OP_FORWARD, true, F1>(g, un, uc, up, kap, slabs, 4, st, &po, nullptr, -1, 16)
                : launch_tiled<R, 32, 8, OP_FORWARD, true, F0>(g, un, uc, up, kap, slabs, 4, st, &po, nullptr, -1, 16);
    if (rc != RTM_OK) return rc;
    return nt ? launch_tiled<R, 2, 32, OP_FORWARD, true, F1>(g, un, uc, up, kap, cols, 2, st, &po, nullptr, -1, 32)
              : launch_tiled<R, 2, 32, OP_FORWARD, true, F0>(g, un, uc, up, kap, cols, 2, st, &po, nullptr, -1, 32);
}

template <int R, int OP = OP_FORWARD>
int launch_interior(const Geo &g, float *un, const float *uc, const float *up, const float *kap, hipStream_t st)
{
    const Region r = halo_region(g.nx, g.ny, g.nz, R);
    const int boxes[1][6] = {{r.wx, g.nx - r.wx, r.hy, g.ny - r.hy, r.hz, g.nz - r.hz}};
    if (vector_path(g, un, uc, up, kap)) {
        const int var = g_opt.interior_variant.load(std::memory_order_relaxed);
        return launch_tiled_variant<R, OP>(var, g, un, uc, up, kap, boxes, 1, st);
    }
    return launch_box_scalar<R, OP>(g, un, uc, up, kap, boxes[0], st);
}

// Every owned cell in one launch: a single box of the tiled kernel (its own tile option) over the
// whole owned block; like the halo call it reads the ghost ring.
// The one-launch call's tile shape: the option, or by radius (6, the default): at radius 4 the 32x8
// tiles (128x8 cells; 343 us for the 512^3 step, 32x16 376 us, 16x16 356 us), at radius 2 the 32x16
// tiles (384^3 coarse step: 216 us, the other shapes 219-258 us).
int whole_variant(int R)
{
    const int v = g_opt.whole_variant.load(std::memory_order_relaxed);
    return v == 6 ? (R == 4 ? 1 : 4) : v;
}

// Settings that rtm_tune_step measured fastest for the one-launch call on grids of one shape on one
// device (tile variant and workgroup order); used while RTM_OPT_WHOLE_VARIANT is 6.  A small table:
// when full, the oldest entry goes.
struct Tuned {
    int dev, nx, ny, nz, R;
    long long py, pz;
    int var, remap;
};
constexpr int kMaxTuned = 32;
std::mutex g_tuned_mu;
Tuned g_tuned[kMaxTuned];
int g_ntuned = 0, g_tuned_next = 0;

bool same_shape(const Tuned &t, int dev, const Geo &g)
{
    return t.dev == dev && t.nx == g.nx && t.ny == g.ny && t.nz == g.nz && t.R == g.R && t.py == g.py && t.pz == g.pz;
}

// The one-launch call's tile variant and workgroup order (-1: the option) for grid g.
void whole_settings(const Geo &g, int R, int &var, int &remap)
{
    var = whole_variant(R);
    remap = -1;
    if (g_opt.whole_variant.load(std::memory_order_relaxed) != 6) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    for (int i = 0; i < g_ntuned; ++i)
        if (same_shape(g_tuned[i], dev, g)) {
            var = g_tuned[i].var;
            remap = g_tuned[i].remap;
            return;
        }
}

void tuned_store(int dev, const Geo &g, int var, int remap)
{
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    for (int i = 0; i < g_ntuned; ++i)
        if (same_shape(g_tuned[i], dev, g)) {
            g_tuned[i].var = var;
            g_tuned[i].remap = remap;
            return;
        }
    const Tuned t = {dev, g.nx, g.ny, g.nz, g.R, g.py, g.pz, var, remap};
    if (g_ntuned < kMaxTuned) {
        g_tuned[g_ntuned++] = t;
    } else {
        g_tuned[g_tuned_next] = t;
        g_tuned_next = (g_tuned_next + 1) % kMaxTuned;
    }
}

template <int R, int OP = OP_FORWARD>
int launch_all(const Geo &g, float *un, const float *uc, const float *up, const float *kap, hipStream_t st)
{
    const int boxes[1][6] = {{0, g.nx, 0, g.ny, 0, g.nz}};
    if (vector_path(g, un, uc, up, kap)) {
        int var, remap;
        whole_settings(g, R, var, remap);
        return launch_tiled_variant<R, OP>(var, g, un, uc, up, kap, boxes, 1, st, nullptr, nullptr, false, remap);
    }
    return launch_box_scalar<R, OP>(g, un, uc, up, kap, boxes[0], st);
}

// Every owned cell with one of the stencil operations, in one launch (the adjoint recursion and the
// gradient accumulation have no exchange to overlap, so they need no halo-first split).
template <int OP>
int launch_whole(const Geo &g, float *un, const float *uc, const float *up, const float *kap, hipStream_t st)
{
    static_assert(OP != OP_ADJOINT, "the adjoint goes through launch_adjoint");
    return g.R == 4 ? launch_all<4, OP>(g, un, uc, up, kap, st) : launch_all<2, OP>(g, un, uc, up, kap, st);
}

// The adjoint step over every owned cell in one launch of the tiled kernel, which forms kappa g mu_a
// from mu_a and kappa as it loads (no weight field).  Tile option: the one-launch call's, except that
// the 128-register tiles (32 x 16, 16 x 32), which the two extra loads per ring element would spill,
// take 16 x 16.  The caller has checked vector_path.
template <int R>
int launch_adjoint(const Geo &g, float *mu_out, const float *mu_a, const float *mu_b, const float *kappa,
                   hipStream_t st)
{
    const int boxes[1][6] = {{0, g.nx, 0, g.ny, 0, g.nz}};
    int var, remap;
    whole_settings(g, R, var, remap);
    if (var == 4 || var == 5) var = 0;
    return launch_tiled_variant<R, OP_ADJOINT>(var, g, mu_out, mu_a, mu_a, mu_b, boxes, 1, st, nullptr, kappa, false,
                                               remap);
}

// Every owned cell in one launch with the ghosts of u_cur read from po.recv (radius 4): the one-launch
// call's tiles and settings, except that the 128-register tiles (32 x 16, 16 x 32), which the slot
// addressing would spill, take 32 x 8.
int launch_whole_slots(const Geo &g, float *un, const float *uc, const float *up, const float *kap, const PackOut &po,
                       hipStream_t st)
{
    const int boxes[1][6] = {{0, g.nx, 0, g.ny, 0, g.nz}};
    int var, remap;
    whole_settings(g, 4, var, remap);
    if (var == 4 || var == 5) var = 1;
    return launch_tiled_variant<4, OP_FORWARD>(var, g, un, uc, up, kap, boxes, 1, st, &po, nullptr, true, remap);
}

bool faces_vec(const Geo &g, const float *u)
{
    return g.R == 4 && (g.nx % 4 == 0) && aligned16(u) && (g.py % 4 == 0) && (g.pz % 4 == 0);
}

int fill_face_offsets(const rtm_grid *gr, long long off[7])
{
    const long long R = gr->radius, nx = gr->nx, ny = gr->ny, nz = gr->nz;
    const long long sz[6] = {R * ny * nz, R * ny * nz, nx * R * nz, nx * R * nz, nx * ny * R, nx * ny * R};
    off[0] = 0;
    for (int f = 0; f < 6; ++f) off[f + 1] = off[f] + sz[f];
    return RTM_OK;
}

bool ranges_overlap(const void *a, long long na, const void *b, long long nb)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    const uintptr_t a1 = a0 + (uintptr_t)na * sizeof(float), b1 = b0 + (uintptr_t)nb * sizeof(float);
    return a0 < b1 && b0 < a1;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Library-owned scratch for the entry points that allocate nothing.  Each device that runs them
// holds one copy of this array until the process ends; host code never passes the array's name to
// a kernel (on the host it stands for the host-side shadow, not the device copy), only the device
// address that hipGetSymbolAddress returns for the current device, cached per device.
// ---------------------------------------------------------------------------------------------
constexpr int kNoAllocMaxChunks = 4096;       // FP64 partial sums: 32 KiB per device
static __device__ __align__(256) double scratch[kNoAllocMaxChunks];

namespace {

std::atomic<double *> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's address of `scratch` (looked up once per device, with it current).
int device_scratch(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RTM_EDEVICE;
    double *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            void *q = nullptr;
            if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return RTM_EDEVICE;
            p = static_cast<double *>(q);
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return RTM_OK;
}

template <int R>
int tune_whole(const Geo &g, float *un, const float *uc, const float *up, const float *kap, int reps, hipStream_t st,
               int &best_var, int &best_remap)
{
    const int boxes[1][6] = {{0, g.nx, 0, g.ny, 0, g.nz}};
    const int vars[5] = {1, 0, 2, 4, 5};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return RTM_ELAUNCH;
    }
    float best = -1.0f;
    int rc = RTM_OK;
    for (int iv = 0; iv < 5 && rc == RTM_OK; ++iv)
        for (int remap = 1; remap >= 0 && rc == RTM_OK; --remap) {
            auto launch = [&] {
                return launch_tiled_variant<R, OP_FORWARD>(vars[iv], g, un, uc, up, kap, boxes, 1, st, nullptr, nullptr,
                                                           false, remap);
            };
            rc = launch();   // warm-up
            if (rc == RTM_OK && hipEventRecord(e0, st) != hipSuccess) rc = RTM_ELAUNCH;
            for (int r = 0; r < reps && rc == RTM_OK; ++r) rc = launch();
            if (rc == RTM_OK && hipEventRecord(e1, st) != hipSuccess) rc = RTM_ELAUNCH;
            float ms = 0.0f;
            if (rc == RTM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = RTM_ELAUNCH;
            if (rc == RTM_OK && (best < 0.0f || ms < best)) {
                best = ms;
                best_var = vars[iv];
                best_remap = remap;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

// =============================================================================================
// extern "C" entry points
// =============================================================================================
extern "C" {

int rtm_abi_version(void) { return RTM_ABI_VERSION; }

const char *rtm_strerror(int status)
{
    switch (status) {
    case RTM_OK: return "ok";
    case RTM_EINVAL: return "invalid argument (null pointer, radius, dimensions, pitches or count)";
    case RTM_EALIAS: return "an output buffer overlaps an input it must not overlap";
    case RTM_ELAUNCH: return "the HIP runtime reported an error at kernel launch";
    case RTM_EDEVICE: return "no HIP device, or the current device is not gfx950";
    default: return "unknown status";
    }
}

int rtm_grid_init(rtm_grid *grid, int32_t nx, int32_t ny, int32_t nz, int32_t radius, int64_t pitch_y,
                  int64_t pitch_z, const float *gx, const float *gy, const float *gz)
{
    if (!grid) return RTM_EINVAL;
    rtm_grid g;
    std::memset(&g, 0, sizeof(g));
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.radius = radius;
    g.pitch_y = pitch_y;
    g.pitch_z = pitch_z;
    g.gx = gx;
    g.gy = gy;
    g.gz = gz;
    // Centred Taylor weights of d2/dx2 on unit spacing (Fornberg 1988), as exact rationals.
    if (radius == 4) {
        const double c[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
        for (int m = 0; m < 5; ++m) g.c[m] = (float)c[m];
    } else if (radius == 2) {
        const double c[3] = {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
        for (int m = 0; m < 3; ++m) g.c[m] = (float)c[m];
    } else {
        return RTM_EINVAL;
    }
    const int st = check_grid(&g);
    if (st != RTM_OK) return st;
    *grid = g;
    return RTM_OK;
}

double rtm_stability_limit(int32_t radius)
{
    double s;
    if (radius == 4)
        s = 205.0 / 72.0 + 2.0 * (8.0 / 5.0 + 1.0 / 5.0 + 8.0 / 315.0 + 1.0 / 560.0);
    else if (radius == 2)
        s = 5.0 / 2.0 + 2.0 * (4.0 / 3.0 + 1.0 / 12.0);
    else
        return 0.0;
    return 2.0 / std::sqrt(3.0 * s);
}

int rtm_stable_dt(int32_t radius, double h, double vmax, double fraction, double *dt)
{
    const double cstar = rtm_stability_limit(radius);
    if (!dt || cstar <= 0.0 || !(h > 0.0) || !(vmax > 0.0) || !(fraction > 0.0)) return RTM_EINVAL;
    *dt = fraction * cstar * h / vmax;
    return RTM_OK;
}

int rtm_injection_weights(int32_t n, const double *v, double dt, double h, float *out)
{
    if (n < 0 || !(dt > 0.0) || !(h > 0.0)) return RTM_EINVAL;
    if (n > 0 && (!v || !out)) return RTM_EINVAL;
    for (int s = 0; s < n; ++s) {
        const double a = v[s] * dt;
        out[s] = (float)(a * a / (h * h * h));
    }
    return RTM_OK;
}

int rtm_sponge_profile(int32_t n, int32_t width, double alpha, float *out)
{
    if (n < 0 || width < 0 || !out) return RTM_EINVAL;
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        if (width > 0) d = std::max(0.0, std::max((double)(width - i), (double)(i - (n - 1 - width))));
        out[i] = (float)std::exp(-(alpha * d) * (alpha * d));
    }
    return RTM_OK;
}

int rtm_ricker(int32_t nsteps, double dt, double fpeak, double t0, float *out)
{
    if (nsteps < 0 || !out) return RTM_EINVAL;
    const double pi = 3.14159265358979323846;
    for (int n = 0; n < nsteps; ++n) {
        const double tau = n * dt - t0;
        const double a = (pi * fpeak * tau) * (pi * fpeak * tau);
        out[n] = (float)((1.0 - 2.0 * a) * std::exp(-a));
    }
    return RTM_OK;
}

int rtm_face_layout(const rtm_grid *grid, int64_t offsets[7])
{
    const int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!offsets) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    for (int f = 0; f < 7; ++f) offsets[f] = off[f];
    return RTM_OK;
}

int64_t rtm_index(const rtm_grid *grid, int32_t i, int32_t j, int32_t k)
{
    if (!grid) return -1;
    const int R = grid->radius;
    return (int64_t)(k + R) * grid->pitch_z + (int64_t)(j + R) * grid->pitch_y + (int64_t)(i + R);
}

static int step_common(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv, const float *kappa)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u_nxt || !u_cur || !u_prv || !kappa) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if (ranges_overlap(u_nxt, tot, u_cur, tot) || ranges_overlap(u_nxt, tot, kappa, tot)) return RTM_EALIAS;
    if (u_nxt != u_prv && ranges_overlap(u_nxt, tot, u_prv, tot)) return RTM_EALIAS;
    return check_device();
}

int rtm_step_halo(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv, const float *kappa,
                  hipStream_t stream)
{
    const Marker mark("rtm_step_halo");
    const int st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    return g.R == 4 ? launch_halo<4>(g, u_nxt, u_cur, u_prv, kappa, stream)
                    : launch_halo<2>(g, u_nxt, u_cur, u_prv, kappa, stream);
}

int rtm_step_interior(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                      const float *kappa, hipStream_t stream)
{
    const Marker mark("rtm_step_interior");
    const int st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    return g.R == 4 ? launch_interior<4>(g, u_nxt, u_cur, u_prv, kappa, stream)
                    : launch_interior<2>(g, u_nxt, u_cur, u_prv, kappa, stream);
}

int rtm_step_whole(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv, const float *kappa,
                   hipStream_t stream)
{
    const Marker mark("rtm_step_whole");
    const int st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    return g.R == 4 ? launch_all<4>(g, u_nxt, u_cur, u_prv, kappa, stream)
                    : launch_all<2>(g, u_nxt, u_cur, u_prv, kappa, stream);
}

int rtm_tune_step(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv, const float *kappa,
                  int32_t reps, int32_t choice[2], hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (reps < 1 || reps > 1000) return RTM_EINVAL;
    if (u_nxt && u_nxt == u_prv) return RTM_EALIAS;     // u_nxt is overwritten: it must be scratch
    st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    int var = -1, remap = -1;
    if (vector_path(g, u_nxt, u_cur, u_prv, kappa)) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return RTM_EDEVICE;
        st = g.R == 4 ? tune_whole<4>(g, u_nxt, u_cur, u_prv, kappa, reps, stream, var, remap)
                      : tune_whole<2>(g, u_nxt, u_cur, u_prv, kappa, reps, stream, var, remap);
        if (st != RTM_OK) return st;
        tuned_store(dev, g, var, remap);
    }
    if (choice) {
        choice[0] = var;
        choice[1] = remap;
    }
    return RTM_OK;
}

int rtm_pack_halo(const rtm_grid *grid, const float *u, float *faces, hipStream_t stream)
{
    const Marker mark("rtm_pack_halo");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u || !faces) return RTM_EINVAL;
    FaceOffsets fo;
    fill_face_offsets(grid, fo.off);
    if (ranges_overlap(faces, fo.off[6], u, padded_total(grid))) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    long long mx = 0;
    for (int f = 0; f < 6; ++f) mx = std::max(mx, fo.off[f + 1] - fo.off[f]);
    const bool narrow = mx < (1ll << 31);     // 32-bit face counters suffice
    if (faces_vec(g, u) && aligned16(faces)) {
        if (narrow)
            hipLaunchKernelGGL(k_pack4<unsigned>, dim3(blocks_for(mx / 4), 6), dim3(kThreads), 0, stream, g, u, faces, fo);
        else
            hipLaunchKernelGGL(k_pack4<long long>, dim3(blocks_for(mx / 4), 6), dim3(kThreads), 0, stream, g, u, faces, fo);
    } else {
        if (narrow)
            hipLaunchKernelGGL(k_pack<unsigned>, dim3(blocks_for(mx), 6), dim3(kThreads), 0, stream, g, u, faces, fo);
        else
            hipLaunchKernelGGL(k_pack<long long>, dim3(blocks_for(mx), 6), dim3(kThreads), 0, stream, g, u, faces, fo);
    }
    return launch_status();
}

int rtm_step_halo_pack(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                       const float *kappa, float *faces, hipStream_t stream)
{
    const Marker mark("rtm_step_halo_pack");
    // the face buffer's own checks first: every argument error is reported before the device check
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!faces) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    const long long tot = padded_total(grid);
    if (ranges_overlap(faces, off[6], u_nxt, tot) || ranges_overlap(faces, off[6], u_cur, tot) ||
        ranges_overlap(faces, off[6], u_prv, tot) || ranges_overlap(faces, off[6], kappa, tot))
        return RTM_EALIAS;
    st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (g.R == 4 && vector_path(g, u_nxt, u_cur, u_prv, kappa) && faces_vec(g, u_nxt) && aligned16(faces)) {
        PackOut po;
        std::memset(&po, 0, sizeof(po));
        po.faces = faces;
        for (int f = 0; f < 6; ++f) po.off[f] = off[f];
        return launch_halo_pack(g, u_nxt, u_cur, u_prv, kappa, po, stream);
    }
    st = rtm_step_halo(grid, u_nxt, u_cur, u_prv, kappa, stream);
    if (st != RTM_OK) return st;
    return rtm_pack_halo(grid, u_nxt, faces, stream);
}

int rtm_step_halo_pack_slots(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                             const float *kappa, const float *const recv[6], float *faces, hipStream_t stream)
{
    const Marker mark("rtm_step_halo_pack_slots");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!faces || !recv) return RTM_EINVAL;
    for (int f = 0; f < 6; ++f)
        if (!recv[f] || !aligned16(recv[f])) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    const long long tot = padded_total(grid);
    if (ranges_overlap(faces, off[6], u_nxt, tot) || ranges_overlap(faces, off[6], u_cur, tot) ||
        ranges_overlap(faces, off[6], u_prv, tot) || ranges_overlap(faces, off[6], kappa, tot))
        return RTM_EALIAS;
    for (int f = 0; f < 6; ++f)   // what this call writes must not be what it reads
        if (ranges_overlap(recv[f], off[f + 1] - off[f], faces, off[6]) ||
            ranges_overlap(recv[f], off[f + 1] - off[f], u_nxt, tot))
            return RTM_EALIAS;
    const Geo g = make_geo(grid);
    if (!(g.R == 4 && vector_path(g, u_nxt, u_cur, u_prv, kappa) && faces_vec(g, u_nxt) && aligned16(faces)))
        return RTM_EINVAL;
    st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    PackOut po;
    po.faces = faces;
    for (int f = 0; f < 6; ++f) {
        po.off[f] = off[f];
        po.recv[f] = recv[f];
    }
    return launch_halo_pack(g, u_nxt, u_cur, u_prv, kappa, po, stream, true);
}

int rtm_step_shell_pack(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *kappa,
                        const float *faces_cur, const float *faces_prv, const float *faces_kappa,
                        const float *const recv[6], float *faces, hipStream_t stream)
{
    const Marker mark("rtm_step_shell_pack");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u_cur || !u_prv || !kappa || !faces || !recv) return RTM_EINVAL;
    for (int f = 0; f < 6; ++f)
        if (!recv[f] || !aligned16(recv[f])) return RTM_EINVAL;
    const bool dense = faces_cur != nullptr;
    if (dense != (faces_prv != nullptr) || dense != (faces_kappa != nullptr)) return RTM_EINVAL;
    if (dense && !(aligned16(faces_cur) && aligned16(faces_prv) && aligned16(faces_kappa))) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    const long long tot = padded_total(grid);
    if (ranges_overlap(faces, off[6], u_cur, tot) || ranges_overlap(faces, off[6], u_prv, tot) ||
        ranges_overlap(faces, off[6], kappa, tot))
        return RTM_EALIAS;
    for (int f = 0; f < 6; ++f)   // what this call writes must not be what it reads
        if (ranges_overlap(recv[f], off[f + 1] - off[f], faces, off[6])) return RTM_EALIAS;
    if (dense && (ranges_overlap(faces_cur, off[6], faces, off[6]) || ranges_overlap(faces_prv, off[6], faces, off[6]) ||
                  ranges_overlap(faces_kappa, off[6], faces, off[6])))
        return RTM_EALIAS;
    const Geo g = make_geo(grid);
    if (!(g.R == 4 && vector_path(g, const_cast<float *>(u_cur), u_cur, u_prv, kappa) && faces_vec(g, u_cur) &&
          aligned16(faces)))
        return RTM_EINVAL;
    st = check_device();
    if (st != RTM_OK) return st;
    PackOut po;
    po.faces = faces;
    for (int f = 0; f < 6; ++f) {
        po.off[f] = off[f];
        po.recv[f] = recv[f];
    }
    return launch_shell_pack(g, u_cur, u_prv, kappa, faces_cur, faces_prv, faces_kappa, po, stream);
}

int rtm_step_whole_slots(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                         const float *kappa, const float *const recv[6], hipStream_t stream)
{
    const Marker mark("rtm_step_whole_slots");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!recv) return RTM_EINVAL;
    for (int f = 0; f < 6; ++f)
        if (!recv[f] || !aligned16(recv[f])) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    const long long tot = padded_total(grid);
    if (!u_nxt || !u_cur || !u_prv || !kappa) return RTM_EINVAL;
    for (int f = 0; f < 6; ++f)   // what this call writes must not be what it reads
        if (ranges_overlap(recv[f], off[f + 1] - off[f], u_nxt, tot)) return RTM_EALIAS;
    const Geo g = make_geo(grid);
    if (!(g.R == 4 && vector_path(g, u_nxt, u_cur, u_prv, kappa) && faces_vec(g, u_nxt))) return RTM_EINVAL;
    st = step_common(grid, u_nxt, u_cur, u_prv, kappa);
    if (st != RTM_OK) return st;
    PackOut po;
    std::memset(&po, 0, sizeof(po));
    for (int f = 0; f < 6; ++f) po.recv[f] = recv[f];
    return launch_whole_slots(g, u_nxt, u_cur, u_prv, kappa, po, stream);
}

int rtm_pack_cells(const rtm_grid *grid, const float *u, const int64_t *idx, int32_t n, float *faces,
                   hipStream_t stream)
{
    const Marker mark("rtm_pack_cells");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (n < 0 || (n > 0 && (!u || !idx || !faces))) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    FaceOffsets fo;
    fill_face_offsets(grid, fo.off);
    if (ranges_overlap(faces, fo.off[6], u, padded_total(grid))) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    hipLaunchKernelGGL(k_pack_cells, dim3(blocks_for(n)), dim3(kThreads), 0, stream, g, u,
                       reinterpret_cast<const long long *>(idx), (int)n, faces, fo);
    return launch_status();
}

int rtm_unpack_halo(const rtm_grid *grid, float *u, const float *const faces[6], hipStream_t stream)
{
    const Marker mark("rtm_unpack_halo");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u || !faces) return RTM_EINVAL;
    long long off[7];
    fill_face_offsets(grid, off);
    FacePtrs fp;
    const long long tot = padded_total(grid);
    for (int f = 0; f < 6; ++f) {
        fp.p[f] = faces[f];
        if (faces[f] && ranges_overlap(faces[f], off[f + 1] - off[f], u, tot)) return RTM_EALIAS;
    }
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    long long mx = 0;
    for (int f = 0; f < 6; ++f) mx = std::max(mx, off[f + 1] - off[f]);
    bool vec = faces_vec(g, u);
    for (int f = 0; f < 6; ++f) vec = vec && (fp.p[f] == nullptr || aligned16(fp.p[f]));
    const bool narrow = mx < (1ll << 31);     // 32-bit face counters suffice
    const bool lines = vec && g.nx % 32 == 0 && g.py == (long long)g.nx + 32 && g.pz % 32 == 0 &&
                       (reinterpret_cast<uintptr_t>(u + (4ll * g.pz + 4ll * g.py + 4)) & 127u) == 0 &&
                       g_opt.unpack_lines.load(std::memory_order_relaxed);
    if (lines) {
        // the x faces as (ny + 1) nz lines of eight float4 each; the y / z faces as before
        const long long items = std::max(8ll * (g.ny + 1) * g.nz, mx / 4);
        if (items < (1ll << 31))
            hipLaunchKernelGGL(k_unpack_lines<unsigned>, dim3(blocks_for(items), 5), dim3(kThreads), 0, stream, g, u,
                               fp);
        else
            hipLaunchKernelGGL(k_unpack_lines<long long>, dim3(blocks_for(items), 5), dim3(kThreads), 0, stream, g,
                               u, fp);
    } else if (vec) {
        if (narrow)
            hipLaunchKernelGGL(k_unpack4<unsigned>, dim3(blocks_for(mx / 4), 6), dim3(kThreads), 0, stream, g, u, fp);
        else
            hipLaunchKernelGGL(k_unpack4<long long>, dim3(blocks_for(mx / 4), 6), dim3(kThreads), 0, stream, g, u, fp);
    } else {
        if (narrow)
            hipLaunchKernelGGL(k_unpack<unsigned>, dim3(blocks_for(mx), 6), dim3(kThreads), 0, stream, g, u, fp);
        else
            hipLaunchKernelGGL(k_unpack<long long>, dim3(blocks_for(mx), 6), dim3(kThreads), 0, stream, g, u, fp);
    }
    return launch_status();
}

int rtm_inject(const rtm_grid *grid, float *u, const int64_t *idx, const float *w, const float *amp, int32_t n,
               hipStream_t stream)
{
    const Marker mark("rtm_inject");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!u || !idx || !w || !amp) return RTM_EINVAL;
    st = check_device();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_inject, dim3(blocks_for(n)), dim3(kThreads), 0, stream, u, padded_total(grid), idx, w, amp,
                       (int)n);
    return launch_status();
}

int rtm_inject_record(const rtm_grid *grid, float *u, const int64_t *src_idx, const float *w, const float *amp,
                      int32_t nsrc, const int64_t *rec_idx, float *out, int32_t nrec, hipStream_t stream)
{
    const Marker mark("rtm_inject_record");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (nsrc < 0 || nrec < 0) return RTM_EINVAL;
    if ((nsrc > 0 && (!u || !src_idx || !w || !amp)) || (nrec > 0 && (!u || !rec_idx || !out))) return RTM_EINVAL;
    if (nsrc == 0 && nrec == 0) return RTM_OK;
    st = check_device();
    if (st != RTM_OK) return st;
    const long long total = padded_total(grid);
    if ((long long)nsrc + nrec <= kInjectRecordOneGroup) {
        hipLaunchKernelGGL(k_inject_record, dim3(1), dim3(kInjectRecordThreads), 0, stream, u, total, src_idx, w, amp,
                           (int)nsrc, rec_idx, out, (int)nrec);
        return launch_status();
    }
    if (nsrc > 0) {
        hipLaunchKernelGGL(k_inject, dim3(blocks_for(nsrc)), dim3(kThreads), 0, stream, u, total, src_idx, w, amp,
                           (int)nsrc);
        st = launch_status();
        if (st != RTM_OK) return st;
    }
    if (nrec > 0) {
        hipLaunchKernelGGL(k_record, dim3(blocks_for(nrec)), dim3(kThreads), 0, stream, u, total, rec_idx, out,
                           (int)nrec);
        st = launch_status();
    }
    return st;
}

int rtm_record(const rtm_grid *grid, const float *u, const int64_t *idx, float *out, int32_t n, hipStream_t stream)
{
    const Marker mark("rtm_record");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!u || !idx || !out) return RTM_EINVAL;
    st = check_device();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_record, dim3(blocks_for(n)), dim3(kThreads), 0, stream, u, padded_total(grid), idx, out,
                       (int)n);
    return launch_status();
}

int rtm_image_accumulate(const rtm_grid *grid, float *image, const float *src, const float *rcv, float weight,
                         hipStream_t stream)
{
    const Marker mark("rtm_image_accumulate");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!image || !src || !rcv) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if (ranges_overlap(image, tot, src, tot) || ranges_overlap(image, tot, rcv, tot)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    const bool nt = (g_opt.tile_flags.load(std::memory_order_relaxed) & FL_NT) != 0;
    if (rows_vec(g) && aligned16(image) && aligned16(src) && aligned16(rcv) && nt)
        hipLaunchKernelGGL((k_image<true, true>), dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image, src, rcv,
                           weight);
    else if (rows_vec(g) && aligned16(image) && aligned16(src) && aligned16(rcv))
        hipLaunchKernelGGL(k_image<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image, src, rcv, weight);
    else
        hipLaunchKernelGGL(k_image<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image, src, rcv, weight);
    return launch_status();
}

int rtm_kappa_from_velocity(const rtm_grid *grid, float *kappa, const float *v, float dt_over_h, hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!kappa || !v) return RTM_EINVAL;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (ranges_overlap(kappa, padded_total(grid), v, n)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (rows_vec(g) && aligned16(kappa) && aligned16(v))
        hipLaunchKernelGGL(k_kappa<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, kappa, v, dt_over_h);
    else
        hipLaunchKernelGGL(k_kappa<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, kappa, v, dt_over_h);
    return launch_status();
}

int rtm_count_nonfinite(const rtm_grid *grid, const float *u, uint32_t *count, hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u || !count) return RTM_EINVAL;
    if (ranges_overlap(count, 1, u, padded_total(grid))) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (rows_vec(g) && aligned16(u))
        hipLaunchKernelGGL(k_count_nonfinite<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, u, count);
    else
        hipLaunchKernelGGL(k_count_nonfinite<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, u, count);
    return launch_status();
}

int rtm_halo_region(const rtm_grid *grid, int32_t widths[3])
{
    const int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!widths) return RTM_EINVAL;
    const Region r = halo_region(grid->nx, grid->ny, grid->nz, grid->radius);
    widths[0] = r.wx;
    widths[1] = r.hy;
    widths[2] = r.hz;
    return RTM_OK;
}

int rtm_adjoint_step(const rtm_grid *grid, float *mu_out, const float *mu_a, const float *mu_b, const float *kappa,
                     float *work, hipStream_t stream)
{
    const Marker mark("rtm_adjoint_step");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!mu_out || !mu_a || !mu_b || !kappa || !work) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if (ranges_overlap(mu_out, tot, mu_a, tot) || ranges_overlap(mu_out, tot, kappa, tot) ||
        ranges_overlap(mu_out, tot, work, tot) || ranges_overlap(work, tot, mu_a, tot) ||
        ranges_overlap(work, tot, mu_b, tot) || ranges_overlap(work, tot, kappa, tot))
        return RTM_EALIAS;
    if (mu_out != mu_b && ranges_overlap(mu_out, tot, mu_b, tot)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (vector_path(g, mu_out, mu_a, mu_b, kappa))
        return g.R == 4 ? launch_adjoint<4>(g, mu_out, mu_a, mu_b, kappa, stream)
                        : launch_adjoint<2>(g, mu_out, mu_a, mu_b, kappa, stream);
    // scalar path: kappa g mu_a into `work` (zero ghosts), then the per-cell update reads it
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_adjoint_weight, dim3(blocks_for(n)), dim3(kThreads), 0, stream, g, work, mu_a, kappa);
    st = launch_status();
    if (st != RTM_OK) return st;
    const int box[6] = {0, g.nx, 0, g.ny, 0, g.nz};
    return g.R == 4 ? launch_box_scalar<4, OP_ADJOINT>(g, mu_out, work, mu_a, mu_b, box, stream)
                    : launch_box_scalar<2, OP_ADJOINT>(g, mu_out, work, mu_a, mu_b, box, stream);
}

int rtm_gradient_accumulate(const rtm_grid *grid, float *grad, const float *u, const float *mu, hipStream_t stream)
{
    const Marker mark("rtm_gradient_accumulate");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!grad || !u || !mu) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if (ranges_overlap(grad, tot, u, tot) || ranges_overlap(grad, tot, mu, tot)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    return launch_whole<OP_GRADIENT>(g, grad, u, mu, grad, stream);
}

int rtm_gradient_accumulate_scaled(const rtm_grid *grid, float *grad, const float *u, const float *w,
                                   hipStream_t stream)
{
    const Marker mark("rtm_gradient_accumulate_scaled");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!grad || !u || !w) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if (ranges_overlap(grad, tot, u, tot) || ranges_overlap(grad, tot, w, tot)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    return launch_whole<OP_GRADIENT_SCALED>(g, grad, u, w, grad, stream);
}

int rtm_scaled_adjoint_factors(const rtm_grid *grid, const float *kappa, const int64_t *idx, int32_t n, float *kg,
                               float *inv_kg, hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!kappa || !idx || (!kg && !inv_kg)) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    if ((kg && ranges_overlap(kg, n, kappa, tot)) || (inv_kg && ranges_overlap(inv_kg, n, kappa, tot)) ||
        (kg && inv_kg && ranges_overlap(kg, n, inv_kg, n)))
        return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    hipLaunchKernelGGL(k_scaled_factors, dim3(blocks_for(n)), dim3(kThreads), 0, stream, g, kappa,
                       reinterpret_cast<const long long *>(idx), (int)n, kg, inv_kg);
    return launch_status();
}

int rtm_record_weighted(const rtm_grid *grid, const float *u, const int64_t *idx, const float *w, float *out,
                        int32_t n, hipStream_t stream)
{
    const Marker mark("rtm_record_weighted");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!u || !idx || !w || !out) return RTM_EINVAL;
    st = check_device();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_record_weighted, dim3(blocks_for(n)), dim3(kThreads), 0, stream, u, padded_total(grid), idx,
                       w, out, (int)n);
    return launch_status();
}

int rtm_velocity_gradient_scaled(const rtm_grid *grid, float *grad_v, const float *G, const float *v,
                                 hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!grad_v || !G || !v) return RTM_EINVAL;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (ranges_overlap(grad_v, n, G, padded_total(grid)) || ranges_overlap(grad_v, n, v, n)) return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (rows_vec(g) && aligned16(grad_v) && aligned16(G) && aligned16(v))
        hipLaunchKernelGGL(k_velocity_gradient_scaled<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, grad_v,
                           G, v);
    else
        hipLaunchKernelGGL(k_velocity_gradient_scaled<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g,
                           grad_v, G, v);
    return launch_status();
}

int rtm_misfit_residual(const float *d, const float *obs, float *resid, int64_t n, double *misfit, hipStream_t stream)
{
    if (n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!d || !obs || !resid || !misfit) return RTM_EINVAL;
    if ((resid != d && ranges_overlap(resid, n, d, n)) || (resid != obs && ranges_overlap(resid, n, obs, n)))
        return RTM_EALIAS;
    const int st = check_device();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_residual, dim3(1), dim3(kReduceThreads), 0, stream, d, obs, resid, (long long)n, misfit);
    return launch_status();
}

int rtm_misfit_residual_chunks(const float *d, const float *obs, float *resid, int64_t n, double *partials,
                               int32_t nchunks, double *misfit, hipStream_t stream)
{
    if (n < 0 || nchunks <= 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!d || !obs || !resid || !misfit || !partials) return RTM_EINVAL;
    if ((resid != d && ranges_overlap(resid, n, d, n)) || (resid != obs && ranges_overlap(resid, n, obs, n)))
        return RTM_EALIAS;
    const long long pf = 2ll * nchunks;               // partials in floats
    if (ranges_overlap(partials, pf, misfit, 2) || ranges_overlap(partials, pf, d, n) ||
        ranges_overlap(partials, pf, obs, n) || ranges_overlap(partials, pf, resid, n))
        return RTM_EALIAS;
    const int st = check_device();
    if (st != RTM_OK) return st;
    const long long chunk = (n + nchunks - 1) / nchunks;
    const long long nb = (n + chunk - 1) / chunk;      // chunks that hold samples (<= nchunks)
    hipLaunchKernelGGL(k_residual_chunks, dim3((unsigned)nb), dim3(kChunkThreads), 0, stream, d, obs, resid,
                       (long long)n, chunk, partials);
    const int s1 = launch_status();
    if (s1 != RTM_OK) return s1;
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(kReduceThreads), 0, stream, partials, (int)nb, misfit);
    return launch_status();
}

int rtm_misfit_residual_chunks_noalloc(const float *d, const float *obs, float *resid, int64_t n, int32_t nchunks,
                                       double *misfit, hipStream_t stream)
{
    if (n < 0 || nchunks <= 0 || nchunks > kNoAllocMaxChunks) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    if (!d || !obs || !resid || !misfit) return RTM_EINVAL;
    if ((resid != d && ranges_overlap(resid, n, d, n)) || (resid != obs && ranges_overlap(resid, n, obs, n)))
        return RTM_EALIAS;
    int st = check_device();
    if (st != RTM_OK) return st;
    double *part = nullptr;
    st = device_scratch(&part);
    if (st != RTM_OK) return st;
    const long long chunk = (n + nchunks - 1) / nchunks;
    const long long nb = (n + chunk - 1) / chunk;      // chunks that hold samples (<= nchunks)
    // every slot the final sum reads (part[0..nb)) is written by the first kernel of this call, so the
    // previous call's contents never leak in and nothing needs clearing
    hipLaunchKernelGGL(k_residual_chunks, dim3((unsigned)nb), dim3(kChunkThreads), 0, stream, d, obs, resid,
                       (long long)n, chunk, part);
    st = launch_status();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(kReduceThreads), 0, stream, part, (int)nb, misfit);
    return launch_status();
}

int rtm_velocity_gradient(const rtm_grid *grid, float *grad_v, const float *grad_kappa, const float *v,
                          float dt_over_h, hipStream_t stream)
{
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!grad_v || !grad_kappa || !v) return RTM_EINVAL;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (ranges_overlap(grad_v, n, grad_kappa, padded_total(grid)) || ranges_overlap(grad_v, n, v, n))
        return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    if (rows_vec(g) && aligned16(grad_v) && aligned16(grad_kappa) && aligned16(v))
        hipLaunchKernelGGL(k_velocity_gradient<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, grad_v,
                           grad_kappa, v, dt_over_h * dt_over_h);
    else
        hipLaunchKernelGGL(k_velocity_gradient<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, grad_v,
                           grad_kappa, v, dt_over_h * dt_over_h);
    return launch_status();
}

int rtm_snapshot_encode(const rtm_grid *grid, const float *u, uint16_t *codes, float *scales, int32_t format,
                        hipStream_t stream)
{
    const Marker mark("rtm_snapshot_encode");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!u || !codes || !scales) return RTM_EINVAL;
    if (format != RTM_SNAP_BF16 && format != RTM_SNAP_F16) return RTM_EINVAL;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    const long long tot = padded_total(grid);
    if (ranges_overlap(codes, (n + 1) / 2, u, tot) || ranges_overlap(scales, grid->nz, u, tot) ||
        ranges_overlap(scales, grid->nz, codes, (n + 1) / 2))
        return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    const bool vec = g.nx % 4 == 0 && aligned16(u + g.R * (g.pz + g.py + 1)) && g.py % 4 == 0 && g.pz % 4 == 0;
    if (vec)
        hipLaunchKernelGGL((k_plane_absmax<true>), dim3(g.nz), dim3(kAbsmaxThreads), 0, stream, g, u, scales);
    else
        hipLaunchKernelGGL((k_plane_absmax<false>), dim3(g.nz), dim3(kAbsmaxThreads), 0, stream, g, u, scales);
    st = launch_status();
    if (st != RTM_OK) return st;
    if (rows_vec(g) && aligned16(u) && aligned8(codes))
        hipLaunchKernelGGL(k_encode<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, u, scales, codes,
                           (int)format);
    else
        hipLaunchKernelGGL(k_encode<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, u, scales, codes,
                           (int)format);
    return launch_status();
}

int rtm_image_accumulate_coded(const rtm_grid *grid, float *image, const uint16_t *codes, const float *scales,
                               int32_t format, const float *rcv, float weight, hipStream_t stream)
{
    const Marker mark("rtm_image_accumulate_coded");
    int st = check_grid(grid);
    if (st != RTM_OK) return st;
    if (!image || !codes || !scales || !rcv) return RTM_EINVAL;
    if (format != RTM_SNAP_BF16 && format != RTM_SNAP_F16) return RTM_EINVAL;
    const long long tot = padded_total(grid);
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (ranges_overlap(image, tot, rcv, tot) || ranges_overlap(image, tot, codes, (n + 1) / 2) ||
        ranges_overlap(image, tot, scales, grid->nz))
        return RTM_EALIAS;
    st = check_device();
    if (st != RTM_OK) return st;
    const Geo g = make_geo(grid);
    const bool nt = (g_opt.tile_flags.load(std::memory_order_relaxed) & FL_NT) != 0;
    if (rows_vec(g) && aligned16(image) && aligned16(rcv) && aligned8(codes) && nt)
        hipLaunchKernelGGL((k_image_coded<true, true>), dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image,
                           codes, scales, (int)format, rcv, weight);
    else if (rows_vec(g) && aligned16(image) && aligned16(rcv) && aligned8(codes))
        hipLaunchKernelGGL(k_image_coded<true>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image, codes,
                           scales, (int)format, rcv, weight);
    else
        hipLaunchKernelGGL(k_image_coded<false>, dim3(row_blocks(g)), dim3(kThreads), 0, stream, g, image, codes,
                           scales, (int)format, rcv, weight);
    return launch_status();
}

int rtm_set_option(int32_t option, int32_t value)
{
    switch (option) {
    case RTM_OPT_INTERIOR_VARIANT:
        if (value < 0 || value > 5) return RTM_EINVAL;
        g_opt.interior_variant.store(value);
        return RTM_OK;
    case RTM_OPT_ZCHUNK:
        if (value < 0) return RTM_EINVAL;
        g_opt.zchunk.store(value);
        return RTM_OK;
    case RTM_OPT_XCD_REMAP:
        g_opt.xcd_remap.store(value ? 1 : 0);
        return RTM_OK;
    case RTM_OPT_HALO_X_WIDTH:
        if (value < 1) return RTM_EINVAL;
        g_opt.halo_x_width.store(value);
        return RTM_OK;
    case RTM_OPT_HALO_Y_WIDTH:
        if (value < 1) return RTM_EINVAL;
        g_opt.halo_y_width.store(value);
        return RTM_OK;
    case RTM_OPT_HALO_Z_WIDTH:
        if (value < 0) return RTM_EINVAL;
        g_opt.halo_z_width.store(value);
        return RTM_OK;
    case RTM_OPT_HALO_VARIANT:
        if (value < 0 || value > 5 || value == 3) return RTM_EINVAL;
        g_opt.halo_variant.store(value);
        return RTM_OK;
    case RTM_OPT_WHOLE_VARIANT:
        if (value < 0 || value > 6 || value == 3) return RTM_EINVAL;
        g_opt.whole_variant.store(value);
        return RTM_OK;
    case RTM_OPT_UNPACK_LINES:
        g_opt.unpack_lines.store(value ? 1 : 0);
        return RTM_OK;
    case RTM_OPT_TILE_FLAGS:
        if (value < 0 || value > 3) return RTM_EINVAL;
        g_opt.tile_flags.store(value);
        return RTM_OK;
    case RTM_OPT_MARKERS:
        if (value < 0 || value > 1) return RTM_EINVAL;
        if (value == 1 && !roctx().push) return RTM_EINVAL;
        g_opt.markers.store(value);
        return RTM_OK;
    default: return RTM_EINVAL;
    }
}

int rtm_get_option(int32_t option)
{
    switch (option) {
    case RTM_OPT_INTERIOR_VARIANT: return g_opt.interior_variant.load();
    case RTM_OPT_ZCHUNK: return g_opt.zchunk.load();
    case RTM_OPT_XCD_REMAP: return g_opt.xcd_remap.load();
    case RTM_OPT_HALO_X_WIDTH: return g_opt.halo_x_width.load();
    case RTM_OPT_HALO_Y_WIDTH: return g_opt.halo_y_width.load();
    case RTM_OPT_HALO_Z_WIDTH: return g_opt.halo_z_width.load();
    case RTM_OPT_HALO_VARIANT: return g_opt.halo_variant.load();
    case RTM_OPT_WHOLE_VARIANT: return g_opt.whole_variant.load();
    case RTM_OPT_UNPACK_LINES: return g_opt.unpack_lines.load();
    case RTM_OPT_TILE_FLAGS: return g_opt.tile_flags.load();
    case RTM_OPT_MARKERS: return g_opt.markers.load();
    default: return RTM_EINVAL;
    }
}

}  // extern "C"
