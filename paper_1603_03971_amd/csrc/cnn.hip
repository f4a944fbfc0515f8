// cnn.hip -- the learned dispersion corrector: a small 3-D CNN on BF16 MFMA with FP32 accumulation,
// its training kernels, and the glue between the coarse-grid wavefield and the network.
//
// Activations are channel-last BF16 volumes with 16 channels and a one-voxel zero halo: element
// (c, i, j, k) of an nx*ny*nz volume lives at (((k+1)(ny+2) + (j+1))(nx+2) + (i+1)) * 16 + c.  A
// 3x3x3 convolution with 16 input and 16 output channels is an implicit GEMM over blocks of 16
// voxels along x: the forward kernel sums two taps per 16x16x32 MFMA with the weights in registers
// and the shifted voxels from a staged input plane (k_conv3d); the weight gradient uses one
// 16x16x16 MFMA per tap with the voxels as the reduction dimension (k_conv3d_wgrad).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "rtm.h"

namespace {

// Rows (waves) per forward-convolution workgroup: 4 or 8 (a build-time choice).
#ifndef RTM_CONV_TY
#define RTM_CONV_TY 4
#endif

constexpr int kC = 16;          // channels

// Elementwise kernels walk their items with a grid-sized stride and 64-bit counters (nblk caps the
// grid), so volumes of more than 2^32 items fit a launch.
__device__ __forceinline__ long long first_item() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long item_stride() { return (long long)gridDim.x * blockDim.x; }
constexpr int kTaps = 27;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

struct Vol {
    int nx, ny, nz;
    __device__ __forceinline__ long long at(int i, int j, int k) const   // padded voxel index
    {
        return ((long long)(k + 1) * (ny + 2) + (j + 1)) * (long long)(nx + 2) + (i + 1);
    }
    __device__ __forceinline__ long long flat(int i, int j, int k) const // compact voxel index
    {
        return ((long long)k * ny + j) * (long long)nx + i;
    }
};

// Padded coarse-grid geometry (the rtm_grid layout): owned cell (i, j, k) of a field.
struct G {
    int nx, ny, nz, R;
    long long py, pz;
    __device__ __forceinline__ long long idx(int i, int j, int k) const
    {
        return (long long)(k + R) * pz + (long long)(j + R) * py + (i + R);
    }
};

// Network input of one voxel from the two levels and the velocity: a = u^n / s, d = (u^n - u^{n-1})
// / s (the difference formed in FP32 before any rounding), m = (v - v_ref) / v_scale.  The pack
// kernel and the first convolution's fused loader both form them here, so they round identically.
__device__ __forceinline__ void input_levels(float uc, float up, float inv, float &a, float &d)
{
    a = uc * inv;
    d = (uc - up) * inv;
}
__device__ __forceinline__ float input_material(float vel, float v_ref, float v_inv) { return (vel - v_ref) * v_inv; }
// Channels 0..7 of the voxel as BF16 (a, d, m a, m d, then zeros).
__device__ __forceinline__ uint4 input_voxel(float a, float d, float m)
{
    return make_uint4((uint32_t)f2bf(a) | ((uint32_t)f2bf(d) << 16),
                      (uint32_t)f2bf(m * a) | ((uint32_t)f2bf(m * d) << 16), 0u, 0u);
}

// What the fused first and last layers read and write besides the activation volumes.
struct Glue {
    G g;                                  // the coarse grid (same nx, ny, nz as the volume)
    const float *u_cur, *u_prv, *vel;     // first layer: the levels and the compact velocity
    float v_ref, v_inv;
    const float *scale;                   // s, on the device
    float *c_cur, *c_prv;                 // last layer: the levels it corrects
    const float *mask;                    // last layer: per-voxel weight of the correction, or null
};

constexpr int kFromVolume = 0, kFromFields = 1;   // where the input plane comes from
constexpr int kToVolume = 0, kToFields = 1;       // where the output goes

// Forward convolution, as MFMAs with M = output channel, N = 16 voxels along x and K = 32: two
// taps of 16 input channels each, D[co][voxel] += sum over the pair's taps and ci of
// W_t[co][ci] X[voxel + tap][ci] (v_mfma_f32_16x16x32_bf16).  The MFMA sums over k, so any mapping of
// (tap, ci) onto a lane's k slots is exact as long as A and B use the same one: here lanes of
// k-group q < 2 carry the pair's first tap, channels 8q..8q+7, and lanes of q >= 2 its second tap,
// channels 8(q-2)..; lane l holds W[co = l % 16][those ci] (A, in registers for the whole launch)
// and X[voxel = l % 16][those ci] (B, one 16-byte LDS read).  Output (16x16 D layout): lane l ends
// with channels 4(l/16)..4(l/16)+3 of voxel l % 16, so the stores of a wave are one contiguous run.
//
// A workgroup of TY waves owns a tile of 64 (x) by TY (y) voxels and marches through a chunk of z
// planes, input plane by input plane: the plane (with a one-voxel rim) is staged in LDS once
// (double buffered, the next plane fetched into registers meanwhile), each of its 16-byte fragments
// is read once and feeds the three output planes it touches (three accumulator sets, rotating),
// and the output plane that has received all three of its input planes is stored.  Per input plane
// and wave: 4 segments x 5 tap pairs (the 9 in-plane taps, the last pair half empty) = 20 LDS reads
// and x 3 output planes = 60 MFMAs.
//
// IN = kFromFields: the first layer of the corrector, with the input volume never written: the
// loader forms each staged voxel from the two levels and the velocity (input_voxel, as the pack
// kernel does) and zero outside the grid, as the volume's halo is.  OUT = kToFields: the last
// layer, whose channels 0 and 1 are applied to the levels in place (as the apply kernel does with
// them) instead of being stored.
template <int TY, int IN, int OUT>
__global__ __launch_bounds__(64 * TY) void k_conv3d(Vol v, int zc, const uint16_t *__restrict__ x,
                                                    const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                    int relu, float *__restrict__ y32, int y32c,
                                                    uint16_t *__restrict__ y16, Glue gl)
{
    constexpr int TX = 64, PX = TX + 2, PY = TY + 2;
    constexpr int PLANE = PX * PY * kC;          // BF16 elements of one staged plane
    constexpr int CHUNKS = PX * PY * 2;          // its 16-byte pieces
    constexpr int NT = 64 * TY;
    constexpr int NCH = (CHUNKS + NT - 1) / NT;
    static_assert(NCH <= 4, "plane pieces per thread");
    __shared__ __align__(16) uint16_t lds[2 * PLANE];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * zc;
    const int z1 = min(v.nz, z0 + zc);
    const int y = y0 + wave;
    const int nseg = min(4, (v.nx - x0) >> 4);
    const long long sy = (long long)(v.nx + 2) * kC;
    const long long sz = sy * (v.ny + 2);

    // in-plane tap positions p = 3 dy + dx (offsets + 1); pair j covers positions 2j and 2j + 1
    // (pair 4: position 8 and nothing).  Lanes of q < 2 take the first, q >= 2 the second.
    const int hi = q >> 1;                       // which tap of the pair this lane carries
    const int ci0 = 8 * (q & 1);
    v8bf wf[3][5];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int pos = 2 * j + hi;
            if (pos < 9) {
                const int t = 9 * dz + pos;
                wf[dz][j] = *reinterpret_cast<const v8bf *>(w + ((t * kC + n) * kC + ci0));
            } else {
                wf[dz][j] = v8bf{};
            }
        }
    // LDS offset (BF16 elements) of this lane's fragment for pair j: its position's row and column
    int poff[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int pos = min(2 * j + hi, 8);      // pair 4, second half: a valid place, zero weights
        const int dy = pos / 3, dx = pos % 3;
        poff[j] = ((wave + dy) * PX + n + dx) * kC + ci0;
    }

    long long g0, g1, g2, g3;
    int l0, l1, l2, l3;
    auto piece = [&](int i, long long &go, int &lo) {
        const int cc = min((int)threadIdx.x + i * NT, CHUNKS - 1);
        const int vox = cc >> 1, r = vox / PX, col = vox - r * PX;
        const int py = min(y0 + r, v.ny + 1), px = min(x0 + col, v.nx + 1);
        go = py * sy + (long long)px * kC + (cc & 1) * 8;
        lo = cc * 8;
    };
    piece(0, g0, l0);
    piece(1, g1, l1);
    piece(2, g2, l2);
    piece(3, g3, l3);
    int4 p0, p1, p2, p3;
    // fused first layer: this thread's (at most two) voxels of the staged plane, their grid cells
    // and the raw operands in flight
    constexpr int NV = (PX * PY + NT - 1) / NT;
    static_assert(NV <= 2, "staged voxels per thread");
    int fi0 = 0, fj0 = 0, fo0 = 0, fi1 = 0, fj1 = 0, fo1 = 0;
    bool fin0 = false, fin1 = false, fok0 = false, fok1 = false;
    float fu0 = 0.f, fp0 = 0.f, fv0 = 0.f, fu1 = 0.f, fp1 = 0.f, fv1 = 0.f;
    float inv = 0.0f;
    if constexpr (IN == kFromFields) {
        auto fvox = [&](int i, int &vi, int &vj, int &vo, bool &vin) {
            const int vv = min((int)threadIdx.x + i * NT, PX * PY - 1);
            const int r = vv / PX, col = vv - r * PX;
            vi = x0 + col - 1;
            vj = y0 + r - 1;
            vo = vv * kC;
            vin = vi >= 0 && vi < v.nx && vj >= 0 && vj < v.ny;
        };
        fvox(0, fi0, fj0, fo0, fin0);
        fvox(1, fi1, fj1, fo1, fin1);
        const float s_ = gl.scale[0];
        inv = s_ > 0.0f ? 1.0f / s_ : 0.0f;
    }
#define FIELD_FETCH1(I, kk)                                                                            \
    {                                                                                                  \
        fok##I = fin##I && (kk) >= 0 && (kk) < v.nz;                                                   \
        if (fok##I) {                                                                                  \
            const long long gp_ = gl.g.idx(fi##I, fj##I, (kk));                                        \
            fu##I = gl.u_cur[gp_];                                                                     \
            fp##I = gl.u_prv[gp_];                                                                     \
            fv##I = gl.vel[v.flat(fi##I, fj##I, (kk))];                                                \
        }                                                                                              \
    }
#define FIELD_STASH1(I, dst)                                                                           \
    {                                                                                                  \
        uint4 d_ = make_uint4(0u, 0u, 0u, 0u);                                                         \
        if (fok##I) {                                                                                  \
            float a_, dd_;                                                                             \
            input_levels(fu##I, fp##I, inv, a_, dd_);                                                  \
            d_ = input_voxel(a_, dd_, input_material(fv##I, gl.v_ref, gl.v_inv));                     \
        }                                                                                              \
        *reinterpret_cast<uint4 *>((dst) + fo##I) = d_;                                                \
        *reinterpret_cast<uint4 *>((dst) + fo##I + 8) = make_uint4(0u, 0u, 0u, 0u);                    \
    }
#define CONV_FETCH(pz)                                                                                 \
    {                                                                                                  \
        if constexpr (IN == kFromVolume) {                                                             \
            const uint16_t *src_ = x + (long long)(pz) * sz;                                           \
            p0 = *reinterpret_cast<const int4 *>(src_ + g0);                                           \
            if constexpr (NCH > 1) p1 = *reinterpret_cast<const int4 *>(src_ + g1);                    \
            if constexpr (NCH > 2) p2 = *reinterpret_cast<const int4 *>(src_ + g2);                    \
            if constexpr (NCH > 3) p3 = *reinterpret_cast<const int4 *>(src_ + g3);                    \
        } else {                                                                                       \
            const int kk_ = (pz) - 1;                                                                  \
            FIELD_FETCH1(0, kk_)                                                                       \
            if constexpr (NV > 1) FIELD_FETCH1(1, kk_)                                                 \
        }                                                                                              \
    }
#define CONV_STASH(buf)                                                                                \
    {                                                                                                  \
        uint16_t *dst_ = lds + (buf) * PLANE;                                                          \
        if constexpr (IN == kFromVolume) {                                                             \
            *reinterpret_cast<int4 *>(dst_ + l0) = p0;                                                 \
            if constexpr (NCH > 1) *reinterpret_cast<int4 *>(dst_ + l1) = p1;                          \
            if constexpr (NCH > 2) *reinterpret_cast<int4 *>(dst_ + l2) = p2;                          \
            if constexpr (NCH > 3) *reinterpret_cast<int4 *>(dst_ + l3) = p3;                          \
        } else {                                                                                       \
            FIELD_STASH1(0, dst_)                                                                      \
            if constexpr (NV > 1) FIELD_STASH1(1, dst_)                                                \
        }                                                                                              \
    }

    float bi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bi[i] = bias ? bias[4 * q + i] : 0.0f;

    // output plane z accumulates in set z % 3; input plane zi feeds outputs zi + 1 (dz = 0), zi (1)
    // and zi - 1 (2); after it, output zi - 1 is complete
    v4f acc[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[a][s] = v4f{0.f, 0.f, 0.f, 0.f};

    // fused last layer: lane l corrects voxel x0 + l of the output plane; its two levels and mask
    // value are loaded when the plane's step starts (fetch_levels) and used when it ends
    const float csc = (OUT == kToFields) ? gl.scale[0] : 0.0f;
    const bool own = (OUT == kToFields) && y < v.ny && (lane >> 4) < nseg;
    float lc = 0.f, lp = 0.f, lm = 0.f, a0 = 0.f, a1 = 0.f;
    long long lg = 0;
    auto fetch_levels = [&](int zo) {
        if (own && zo >= z0) {
            lg = gl.g.idx(x0 + lane, y, zo);
            lc = gl.c_cur[lg];
            lp = gl.c_prv[lg];
            lm = gl.mask ? gl.mask[v.flat(x0 + lane, y, zo)] : 1.0f;
        }
    };
    auto apply_levels = [&](int zo) {
        if (own && zo >= z0) {
            const float sv = gl.mask ? csc * lm : csc;
            gl.c_cur[lg] = __builtin_fmaf(sv, a0, lc);
            gl.c_prv[lg] = __builtin_fmaf(sv, a0 - a1, lp);
        }
    };
    auto store = [&](const v4f *o, int zo) {
        if (y >= v.ny || zo < z0) return;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (s >= nseg) break;
            const int xv = x0 + 16 * s + n;
            float r[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                r[i] = o[s][i] + bi[i];
                if (relu) r[i] = fmaxf(r[i], 0.0f);
            }
            if constexpr (OUT == kToFields) {
                // channels 0 and 1 of segment s sit in lanes 0..15 (q = 0); lane l applies them to
                // voxel x0 + l (segment l / 16, position l % 16), so move them there
                const float c0 = __shfl(r[0], n), c1 = __shfl(r[1], n);
                if ((lane >> 4) == s) {
                    a0 = c0;
                    a1 = c1;
                }
                continue;
            }
            if (y16) {
                uint2 pk;
                pk.x = (uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16);
                pk.y = (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16);
                *reinterpret_cast<uint2 *>(y16 + v.at(xv, y, zo) * kC + 4 * q) = pk;
            }
            if (y32) {
                const long long o32 = v.flat(xv, y, zo) * y32c;
                if (y32c == kC) {
                    *reinterpret_cast<float4 *>(y32 + o32 + 4 * q) = make_float4(r[0], r[1], r[2], r[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (4 * q + i < y32c) y32[o32 + 4 * q + i] = r[i];
                }
            }
        }
    };

    // one input plane (staged in buffer `buf`) into the three accumulator sets; A0, A1, A2 are the
    // sets of outputs zi + 1, zi, zi - 1 (compile-time, so the accumulators stay in registers)
    auto plane = [&](auto A0, auto A1, auto A2, int buf) {
        const uint16_t *base = lds + buf * PLANE;
        v8bf cur[4], nxt[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) cur[s] = *reinterpret_cast<const v8bf *>(base + poff[0] + s * 16 * kC);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j + 1 < 5) {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    nxt[s] = *reinterpret_cast<const v8bf *>(base + poff[j + 1] + s * 16 * kC);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc[A0][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[0][j], cur[s], acc[A0][s], 0, 0, 0);
                acc[A1][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[1][j], cur[s], acc[A1][s], 0, 0, 0);
                acc[A2][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[2][j], cur[s], acc[A2][s], 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) cur[s] = nxt[s];
        }
    };

    // input planes zi = z0 - 1 .. z1 (padded index zi + 1); plane k of the march sits in buffer k & 1
    CONV_FETCH(z0)
    CONV_STASH(0)
    CONV_FETCH(z0 + 1)
    __syncthreads();
    const int nin = z1 - z0 + 2;
    auto step = [&](auto R, int k) {
        // input plane zi = z0 - 1 + k; output plane z accumulates in set (z - z0 + 2) % 3, so with
        // r = k % 3 (compile-time R): output zi + 1 in set (r + 2) % 3, zi in (r + 1) % 3, zi - 1 in r
        constexpr int r = decltype(R)::value;
        constexpr int setP = (r + 2) % 3;
        constexpr int set0 = (r + 1) % 3;
        constexpr int setM = r;
        const int buf = k & 1;
        if constexpr (OUT == kToFields) fetch_levels(z0 - 2 + k);
        plane(std::integral_constant<int, setP>{}, std::integral_constant<int, set0>{},
              std::integral_constant<int, setM>{}, buf);
        if (k + 1 < nin) {
            CONV_STASH(buf ^ 1)
            CONV_FETCH(min(z0 + k + 2, v.nz + 1))
        }
        store(acc[setM], z0 - 2 + k);           // output zi - 1 is complete
        if constexpr (OUT == kToFields) apply_levels(z0 - 2 + k);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[setM][s] = v4f{0.f, 0.f, 0.f, 0.f};
        __syncthreads();
    };
    int k = 0;
    for (; k + 3 <= nin; k += 3) {
        step(std::integral_constant<int, 0>{}, k);
        step(std::integral_constant<int, 1>{}, k + 1);
        step(std::integral_constant<int, 2>{}, k + 2);
    }
    if (k < nin) step(std::integral_constant<int, 0>{}, k);
    if (k + 1 < nin) step(std::integral_constant<int, 1>{}, k + 1);
#undef CONV_FETCH
#undef CONV_STASH
#undef FIELD_FETCH1
#undef FIELD_STASH1
}

// Weight gradient.  dw[t][co][ci] += sum over voxels of dz[voxel][co] x[voxel + tap][ci], as MFMAs
// with M = output channel, N = input channel and K = 16 voxels along x.  A wave accumulates a row
// segment for all 27 taps, the workgroup's four waves add their partial sums in LDS, and one atomic
// add per weight and workgroup goes to global memory.  db[co] += sum of dz[voxel][co].
// FIXED: the summation order is fixed.  The four waves add their sums into LDS one after another
// (instead of all at once), the bias sums of a wave's four lanes per channel meet in a fixed
// order, and the workgroup writes its partial sums to its own slot of `part` (kWgradSlot floats:
// the weights, then the biases) for k_wgrad_reduce, instead of adding them with global atomics.
constexpr int kWgradSlot = kTaps * kC * kC + kC;

template <bool FIXED>
__global__ __launch_bounds__(256) void k_conv3d_wgrad(Vol v, const uint16_t *__restrict__ x,
                                                      const float *__restrict__ dz, float *__restrict__ dw,
                                                      float *__restrict__ db, float *__restrict__ part)
{
    __shared__ float red[kTaps * kC * kC];
    __shared__ float redb[kC];
    for (int t = threadIdx.x; t < kTaps * kC * kC; t += 256) red[t] = 0.0f;
    if (threadIdx.x < kC) redb[threadIdx.x] = 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j = blockIdx.y * 4 + wave;
    const int k = blockIdx.z;
    const int m = lane & 15, q = lane >> 4;
    v4f acc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    if (j < v.ny) {
        for (int x0 = blockIdx.x * 64; x0 < min(v.nx, blockIdx.x * 64 + 64); x0 += 16) {
            // A[co = m][vox = 4q + i] = dz[x0 + 4q + i][m]
            v4s a;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float d = dz[v.flat(x0 + 4 * q + i, j, k) * kC + m];
                bsum += d;
                a[i] = (short)f2bf(d);
            }
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int tz = t / 9 - 1, ty = (t / 3) % 3 - 1, tx = t % 3 - 1;
                // B[vox = 4q + i][ci = m] = x[(x0 + 4q + i) + tap][m]
                v4s bb;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    bb[i] = (short)x[v.at(x0 + 4 * q + i + tx, j + ty, k + tz) * kC + m];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[t], 0, 0, 0);
            }
        }
    }
    // D[co = 4q + i][ci = m]: each lane of a wave owns distinct weights
    if constexpr (FIXED) {
        // one wave per phase: its lanes own distinct weights, so each LDS address takes exactly one
        // (uncontended) atomic add per phase, in wave order
#pragma unroll 1
        for (int w = 0; w < 4; ++w) {
            if (wave == w && j < v.ny) {
#pragma unroll
                for (int t = 0; t < kTaps; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) atomicAdd(&red[(t * kC + 4 * q + i) * kC + m], acc[t][i]);
                const float b = ((__shfl(bsum, m) + __shfl(bsum, m + 16)) + __shfl(bsum, m + 32)) + __shfl(bsum, m + 48);
                if (q == 0) atomicAdd(&redb[m], b);
            }
            __syncthreads();
        }
        const long long slot =
            ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        float *dst = part + slot * kWgradSlot;
        for (int t = threadIdx.x; t < kTaps * kC * kC; t += 256) dst[t] = red[t];
        if (threadIdx.x < kC) dst[kTaps * kC * kC + threadIdx.x] = redb[threadIdx.x];
    } else {
        if (j < v.ny) {
#pragma unroll
            for (int t = 0; t < kTaps; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) atomicAdd(&red[(t * kC + 4 * q + i) * kC + m], acc[t][i]);
            atomicAdd(&redb[m], bsum);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kTaps * kC * kC; t += 256) atomicAdd(&dw[t], red[t]);
        if (threadIdx.x < kC) atomicAdd(&db[threadIdx.x], redb[threadIdx.x]);
    }
}

// dw += the sum of the slots' weights and db += their biases, in a fixed order: a workgroup takes 64
// values; its wave w sums the slots w, w + 16, w + 32, ... in slot order (lane l reads value l: 256
// contiguous bytes per slot), and the 16 group sums are then added in group order.
constexpr int kReduceGroups = 16;

__global__ __launch_bounds__(64 * kReduceGroups) void k_wgrad_reduce(const float *__restrict__ part, long long nslot,
                                                                     float *__restrict__ dw, float *__restrict__ db)
{
    __shared__ float grp[kReduceGroups][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (t < kWgradSlot)
        for (long long b = w; b < nslot; b += kReduceGroups) s += part[b * kWgradSlot + t];
    grp[w][lane] = s;
    __syncthreads();
    if (w == 0 && t < kWgradSlot) {
        float tot = grp[0][lane];
        for (int i = 1; i < kReduceGroups; ++i) tot += grp[i][lane];
        if (t < kTaps * kC * kC)
            dw[t] += tot;
        else
            db[t - kTaps * kC * kC] += tot;
    }
}

// dz = dy * (y > 0) for a ReLU layer (relu = 0: dz = dy), over the channels < cmask (others 0);
// written as FP32 (compact) and as BF16 with a zero halo for the data-gradient convolution.
__global__ __launch_bounds__(256) void k_relu_backward(Vol v, const float *__restrict__ y, const float *__restrict__ dy,
                                                       int relu, int cmask, float *__restrict__ dz32,
                                                       uint16_t *__restrict__ dz16)
{
    const long long n = (long long)v.nx * v.ny * v.nz * kC;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int c = (int)(t % kC);
        const long long vox = t / kC;
        const int i = (int)(vox % v.nx);
        const int jj = (int)((vox / v.nx) % v.ny);
        const int kk = (int)(vox / ((long long)v.nx * v.ny));
        float d = c < cmask ? dy[t] : 0.0f;
        if (relu && !(y[t] > 0.0f)) d = 0.0f;
        dz32[t] = d;
        dz16[v.at(i, jj, kk) * kC + c] = f2bf(d);
    }
}

// Output-layer gradient of L = 1/2 sum over voxels and channels < cmask of w (out - target)^2 with
// w = weight * mask[voxel] (mask optional): dz = w (out - target) on those channels (others 0), FP32
// compact and BF16 with a zero halo; L is added into loss[0].
__global__ __launch_bounds__(256) void k_loss_grad(Vol v, const float *__restrict__ out, const float *__restrict__ tgt,
                                                   int cmask, float weight, const float *__restrict__ mask,
                                                   float *__restrict__ dz32, uint16_t *__restrict__ dz16,
                                                   double *__restrict__ loss)
{
    const long long n = (long long)v.nx * v.ny * v.nz * kC;
    double part = 0.0;                         // this thread's share of L
    for (long long t = first_item(); t < n; t += item_stride()) {
        float d = 0.0f;
        const int c = (int)(t % kC);
        const long long vox = t / kC;
        const int i = (int)(vox % v.nx);
        const int jj = (int)((vox / v.nx) % v.ny);
        const int kk = (int)(vox / ((long long)v.nx * v.ny));
        const float wv = mask ? weight * mask[vox] : weight;
        if (c < cmask) d = out[t] - tgt[t];
        dz32[t] = wv * d;
        dz16[v.at(i, jj, kk) * kC + c] = f2bf(wv * d);
        d *= sqrtf(wv);                        // the loss term is wv d^2 / 2
        part += 0.5 * (double)d * (double)d;
    }
    if (!loss) return;
    __shared__ double red[256];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// w_t[t'][ci][co] = w[26 - t'][co][ci]: the weights of the data-gradient convolution.
__global__ void k_weight_flip(const uint16_t *__restrict__ w, uint16_t *__restrict__ wt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kTaps * kC * kC) return;
    const int tap = t / (kC * kC), a = (t / kC) % kC, b = t % kC;
    wt[t] = w[((kTaps - 1 - tap) * kC + b) * kC + a];
}

// Adam (Kingma & Ba 2014) on FP32 master weights; also writes the BF16 copy used by the kernels.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t *__restrict__ p16)
{
    for (long long t = first_item(); t < n; t += item_stride()) {
        const float gt = g[t];
        const float a = b1 * m1[t] + (1.0f - b1) * gt;
        const float b = b2 * m2[t] + (1.0f - b2) * gt * gt;
        m1[t] = a;
        m2[t] = b;
        const float val = p[t] - lr * (a / c1) / (sqrtf(b / c2) + eps);
        p[t] = val;
        if (p16) p16[t] = f2bf(val);
    }
}

__global__ void k_to_bf16(const float *__restrict__ a, uint16_t *__restrict__ b, int n)
{
    for (long long t = first_item(); t < n; t += item_stride()) b[t] = f2bf(a[t]);
}

// ---------------------------------------------------------------------------------------------
// Glue between the coarse-grid wavefield (padded rtm_grid layout) and the network
// ---------------------------------------------------------------------------------------------

G make_g(const rtm_grid *gr) { return G{gr->nx, gr->ny, gr->nz, gr->radius, gr->pitch_y, gr->pitch_z}; }

// The geometry checks of the propagator calls: sizes, radius and pitches consistent.
bool grid_ok(const rtm_grid *gr)
{
    if (!gr || (gr->radius != 2 && gr->radius != 4)) return false;
    const int R = gr->radius;
    if (gr->nx < 2 * R || gr->ny < 2 * R || gr->nz < 2 * R) return false;
    return gr->pitch_y >= (int64_t)gr->nx + 2 * R && gr->pitch_z >= gr->pitch_y * ((int64_t)gr->ny + 2 * R);
}

// Network input: channel 0 = a = u^n / s, 1 = d = (u^n - u^{n-1}) / s, 2 = m a, 3 = m d with the
// material m = (v - v_ref) / v_scale, others 0; s is read from the device (scale[0]); BF16,
// channel-last with a zero halo.  The difference of the two levels, about a tenth of either, is
// formed in FP32 before the rounding: rounding the levels separately would leave it with a few per
// cent of error.  Every channel vanishes where the wavefield does, so a bias-free network maps a
// zero state to a zero correction.  noise (optional, [voxel][2]) is added to a and d
// (training-time augmentation).
__global__ __launch_bounds__(256) void k_pack_input(G g, Vol v, const float *__restrict__ u_cur,
                                                    const float *__restrict__ u_prv, const float *__restrict__ vel,
                                                    float v_ref, float v_inv, const float *__restrict__ scale,
                                                    const float *__restrict__ noise, uint16_t *__restrict__ x)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int i = (int)(t % g.nx);
        const int j = (int)((t / g.nx) % g.ny);
        const int k = (int)(t / ((long long)g.nx * g.ny));
        const float s = scale[0];
        const float inv = s > 0.0f ? 1.0f / s : 0.0f;
        const long long p = g.idx(i, j, k);
        uint16_t *o = x + v.at(i, j, k) * kC;
        float a, d;
        input_levels(u_cur[p], u_prv[p], inv, a, d);
        if (noise) {
            a += noise[2 * t];
            d += noise[2 * t + 1];
        }
        const float m = input_material(vel[t], v_ref, v_inv);
        // the whole 32-byte voxel in two 16-byte stores (a partial store would leave lines to merge)
        reinterpret_cast<uint4 *>(o)[0] = input_voxel(a, d, m);
        reinterpret_cast<uint4 *>(o)[1] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// Apply the correction (out: [voxel][oc], in the input's level-and-difference form): u^n += s o0 and
// u^n - u^{n-1} += s o1, i.e. u^{n-1} += s (o0 - o1), on owned cells; s times mask[voxel] if a mask
// is given.
__global__ __launch_bounds__(256) void k_apply_correction(G g, float *u_cur, float *u_prv, const float *__restrict__ out,
                                                          int oc, const float *__restrict__ mask,
                                                          const float *__restrict__ scale)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int i = (int)(t % g.nx);
        const int j = (int)((t / g.nx) % g.ny);
        const int k = (int)(t / ((long long)g.nx * g.ny));
        const float s = mask ? scale[0] * mask[t] : scale[0];
        const long long p = g.idx(i, j, k);
        const float o0 = out[t * oc + 0], o1 = out[t * oc + 1];
        u_cur[p] = __builtin_fmaf(s, o0, u_cur[p]);
        u_prv[p] = __builtin_fmaf(s, o0 - o1, u_prv[p]);
    }
}

// Training target in the input's form: channel 0 = (ref^n - u^n) / s, channel 1 =
// ((ref^n - ref^{n-1}) - (u^n - u^{n-1})) / s, minus the input noise if any (the network is then asked
// to remove it); FP32 channel-last, other channels 0.
__global__ __launch_bounds__(256) void k_target(G g, const float *__restrict__ ref_cur, const float *__restrict__ ref_prv,
                                                const float *__restrict__ u_cur, const float *__restrict__ u_prv,
                                                const float *__restrict__ scale, const float *__restrict__ noise,
                                                float *__restrict__ tgt)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int i = (int)(t % g.nx);
        const int j = (int)((t / g.nx) % g.ny);
        const int k = (int)(t / ((long long)g.nx * g.ny));
        const float s = scale[0];
        const float inv = s > 0.0f ? 1.0f / s : 0.0f;
        const long long p = g.idx(i, j, k);
        float *o = tgt + t * kC;
        const float rc = ref_cur[p], uc = u_cur[p];
        o[0] = (rc - uc) * inv;
        o[1] = ((rc - ref_prv[p]) - (uc - u_prv[p])) * inv;
        if (noise) {
            o[0] -= noise[2 * t];
            o[1] -= noise[2 * t + 1];
        }
    #pragma unroll
        for (int c = 2; c < kC; ++c) o[c] = 0.0f;
    }
}

// Fine -> coarse restriction.  Injection: coarse (i, j, k) takes fine (2i, 2j, 2k).  Full weighting:
// the separable (1/4, 1/2, 1/4) average of the 27 fine cells around it (ghost cells of the fine field
// enter at the boundary), which preserves integrals: a fine point source of weight 1/h^3 becomes a
// coarse one of weight 1/(2h)^3.
__global__ __launch_bounds__(256) void k_restrict(G f, G c, const float *__restrict__ uf, float *__restrict__ uc,
                                                  int full)
{
    const long long n = (long long)c.nx * c.ny * c.nz;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int i = (int)(t % c.nx);
        const int j = (int)((t / c.nx) % c.ny);
        const int k = (int)(t / ((long long)c.nx * c.ny));
        const long long p = f.idx(2 * i, 2 * j, 2 * k);
        if (!full) {
            uc[c.idx(i, j, k)] = uf[p];
            continue;
        }
        const float w[3] = {0.25f, 0.5f, 0.25f};
        float acc = 0.0f;
        for (int a = 0; a < 3; ++a) {
            float sy = 0.0f;
            for (int b = 0; b < 3; ++b) {
                const float *r = uf + p + (long long)(a - 1) * f.pz + (long long)(b - 1) * f.py;
                const float sx = __builtin_fmaf(w[2], r[1], __builtin_fmaf(w[1], r[0], w[0] * r[-1]));
                sy = __builtin_fmaf(w[b], sx, sy);
            }
            acc = __builtin_fmaf(w[a], sy, acc);
        }
        uc[c.idx(i, j, k)] = acc;
    }
}

// Prolongation, the transpose of full weighting up to a factor 8: fine cell (I, J, K) takes, along each
// axis, coarse cell I/2 for even I and the mean of coarse cells (I-1)/2 and (I+1)/2 for odd I (trilinear
// interpolation between coincident cells; the last odd fine cell reads the coarse ghost layer).
__global__ __launch_bounds__(256) void k_prolong(G c, G f, const float *__restrict__ uc, float *__restrict__ uf)
{
    const long long n = (long long)f.nx * f.ny * f.nz;
    for (long long t = first_item(); t < n; t += item_stride()) {
        const int I = (int)(t % f.nx);
        const int J = (int)((t / f.nx) % f.ny);
        const int K = (int)(t / ((long long)f.nx * f.ny));
        const int i0 = I >> 1, j0 = J >> 1, k0 = K >> 1;
        const int ni = (I & 1) ? 2 : 1, nj = (J & 1) ? 2 : 1, nk = (K & 1) ? 2 : 1;
        float acc = 0.0f;
        for (int a = 0; a < nk; ++a) {
            float sy = 0.0f;
            for (int b = 0; b < nj; ++b) {
                const float *r = uc + c.idx(i0, j0 + b, k0 + a);
                sy += (ni == 2) ? 0.5f * (r[0] + r[1]) : r[0];
            }
            acc += (nj == 2) ? 0.5f * sy : sy;
        }
        uf[f.idx(I, J, K)] = (nk == 2) ? 0.5f * acc : acc;
    }
}

// max |u| over owned cells into out[0] (the corrector's per-application scale): workgroups stride
// over the rows, each thread over a row's cells, and the workgroup maxima are combined with an
// integer atomic max on the bit patterns (non-negative floats order like their bits), so the result
// does not depend on scheduling.
__global__ void k_zero1(float *out) { out[0] = 0.0f; }

// max |u| over the owned cells into out[0] (zeroed by k_zero1 first): a grid-stride walk over the
// cells, x fastest, with four loads in flight per thread, then a wave-shuffle and LDS reduction per
// workgroup and one atomic max of the bit pattern (ordered like the value for non-negative floats).
// I is the index type: 32-bit when the cell count allows.
template <typename I>
__global__ __launch_bounds__(256) void k_absmax_cells(G g, const float *__restrict__ u, float *out)
{
    const I n = (I)g.nx * (I)g.ny * (I)g.nz;
    const I stride = (I)gridDim.x * 256;
    float mx = 0.0f;
    for (I t0 = (I)blockIdx.x * 256 + threadIdx.x; t0 < n; t0 += 4 * stride) {
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const I t = t0 + (I)q * stride;
            v[q] = 0.0f;
            if (t < n) {
                const I r = t / (I)g.nx;
                const int i = (int)(t - r * (I)g.nx);
                const int k = (int)(r / (I)g.ny), j = (int)(r - (I)k * (I)g.ny);
                v[q] = u[g.idx(i, j, k)];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) mx = fmaxf(mx, fabsf(v[q]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        atomicMax(reinterpret_cast<int *>(out), __float_as_int(mx));
    }
}

int status() { return hipGetLastError() == hipSuccess ? RTM_OK : RTM_ELAUNCH; }

// Whether the byte ranges [a, a + na) and [b, b + nb) overlap.
bool bytes_overlap(const void *a, long long na, const void *b, long long nb)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + (uintptr_t)nb && b0 < a0 + (uintptr_t)na;
}

// The kernels are built for gfx950 only: the current device is checked once per device.
std::atomic<int> g_cnn_dev[64];   // 0 unknown, 1 gfx950, -1 other

int device_ok()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RTM_EDEVICE;
    int st = g_cnn_dev[dev].load(std::memory_order_relaxed);
    if (st == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RTM_EDEVICE;
        st = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        g_cnn_dev[dev].store(st, std::memory_order_relaxed);
    }
    return st == 1 ? RTM_OK : RTM_EDEVICE;
}

#define CNN_CHECK_DEVICE()                                                                             \
    do {                                                                                               \
        const int dst_ = device_ok();                                                                  \
        if (dst_ != RTM_OK) return dst_;                                                               \
    } while (0)
// Workgroups for n items; the elementwise kernels stride by the grid beyond the cap, so volumes of
// more than 2^32 items fit one launch dimension.
unsigned nblk(long long n, int t = 256) { return (unsigned)std::min<long long>((n + t - 1) / t, 1ll << 20); }

bool vol_ok(int nx, int ny, int nz) { return nx > 0 && ny > 0 && nz > 0 && nx % 16 == 0; }

// Forward convolution launch: tiles of 64 x TY voxels, z cut into chunks so that there are about
// 2048 workgroups (several per CU) without chunks thinner than needed.
template <int IN, int OUT>
int launch_conv(const Vol &v, const uint16_t *x, const uint16_t *w, const float *bias, int relu, float *y32, int y32c,
                uint16_t *y16, const Glue &gl, hipStream_t stream)
{
    constexpr int TY = RTM_CONV_TY;
    const long long tiles = (long long)((v.nx + 63) / 64) * ((v.ny + TY - 1) / TY);
    long long chunks = (2048 + tiles - 1) / tiles;
    if (chunks > v.nz) chunks = v.nz;
    const int zc = (int)((v.nz + chunks - 1) / chunks);
    const int nzc = (v.nz + zc - 1) / zc;
    hipLaunchKernelGGL((k_conv3d<TY, IN, OUT>), dim3((v.nx + 63) / 64, (v.ny + TY - 1) / TY, nzc), dim3(64 * TY), 0,
                       stream, v, zc, x, w, bias, relu ? 1 : 0, y32, y32c, y16, gl);
    return status();
}

}  // namespace

extern "C" {

int rtm_cnn_conv3d(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const uint16_t *w, const float *bias,
                   int32_t relu, float *y32, int32_t y32_channels, uint16_t *y16, hipStream_t stream)
{
    if (!vol_ok(nx, ny, nz) || !x || !w || (!y32 && !y16)) return RTM_EINVAL;
    if (y32 && (y32_channels < 1 || y32_channels > kC)) return RTM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(x) & 15u) || (reinterpret_cast<uintptr_t>(w) & 15u)) return RTM_EINVAL;
    if ((y16 && (reinterpret_cast<uintptr_t>(y16) & 7u)) || (y32 && (reinterpret_cast<uintptr_t>(y32) & 15u)))
        return RTM_EINVAL;
    if ((const void *)y16 == (const void *)x) return RTM_EALIAS;
    CNN_CHECK_DEVICE();
    Glue gl;
    std::memset(&gl, 0, sizeof(gl));
    return launch_conv<kFromVolume, kToVolume>(Vol{nx, ny, nz}, x, w, bias, relu, y32, y32_channels, y16, gl, stream);
}

int rtm_cnn_conv3d_first(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *velocity,
                         float v_ref, float v_scale, const float *scale, const uint16_t *w, const float *bias,
                         int32_t relu, uint16_t *y16, hipStream_t stream)
{
    if (!grid_ok(grid) || !vol_ok(grid->nx, grid->ny, grid->nz)) return RTM_EINVAL;
    if (!u_cur || !u_prv || !velocity || !scale || !w || !y16 || !(v_scale > 0.0f)) return RTM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(w) & 15u) || (reinterpret_cast<uintptr_t>(y16) & 7u)) return RTM_EINVAL;
    CNN_CHECK_DEVICE();
    Glue gl;
    std::memset(&gl, 0, sizeof(gl));
    gl.g = make_g(grid);
    gl.u_cur = u_cur;
    gl.u_prv = u_prv;
    gl.vel = velocity;
    gl.v_ref = v_ref;
    gl.v_inv = 1.0f / v_scale;
    gl.scale = scale;
    return launch_conv<kFromFields, kToVolume>(Vol{grid->nx, grid->ny, grid->nz}, nullptr, w, bias, relu, nullptr, 0,
                                               y16, gl, stream);
}

int rtm_cnn_conv3d_apply(const rtm_grid *grid, const uint16_t *x, const uint16_t *w, const float *bias, int32_t relu,
                         float *u_cur, float *u_prv, const float *mask, const float *scale, hipStream_t stream)
{
    if (!grid_ok(grid) || !vol_ok(grid->nx, grid->ny, grid->nz)) return RTM_EINVAL;
    if (!x || !w || !u_cur || !u_prv || !scale || u_cur == u_prv) return RTM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(x) & 15u) || (reinterpret_cast<uintptr_t>(w) & 15u)) return RTM_EINVAL;
    CNN_CHECK_DEVICE();
    Glue gl;
    std::memset(&gl, 0, sizeof(gl));
    gl.g = make_g(grid);
    gl.scale = scale;
    gl.c_cur = u_cur;
    gl.c_prv = u_prv;
    gl.mask = mask;
    return launch_conv<kFromVolume, kToFields>(Vol{grid->nx, grid->ny, grid->nz}, x, w, bias, relu, nullptr, 0,
                                               nullptr, gl, stream);
}

int rtm_cnn_conv3d_wgrad(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const float *dz, float *dw, float *db,
                         hipStream_t stream)
{
    if (!vol_ok(nx, ny, nz) || !x || !dz || !dw || !db) return RTM_EINVAL;
    const Vol v{nx, ny, nz};
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_conv3d_wgrad<false>, dim3((nx + 63) / 64, (ny + 3) / 4, nz), dim3(256), 0, stream, v, x, dz, dw,
                       db, nullptr);
    return status();
}

int64_t rtm_cnn_wgrad_partials(int32_t nx, int32_t ny, int32_t nz)
{
    if (!vol_ok(nx, ny, nz)) return RTM_EINVAL;
    return (int64_t)((nx + 63) / 64) * ((ny + 3) / 4) * nz * kWgradSlot;
}

int rtm_cnn_conv3d_wgrad_ordered(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const float *dz, float *dw,
                                 float *db, float *partials, int64_t partials_len, hipStream_t stream)
{
    if (!vol_ok(nx, ny, nz) || !x || !dz || !dw || !db || !partials) return RTM_EINVAL;
    const int64_t need = rtm_cnn_wgrad_partials(nx, ny, nz);
    if (partials_len < need) return RTM_EINVAL;
    const long long pb = (long long)need * 4;
    const long long vox = (long long)nx * ny * nz, pvox = (long long)(nx + 2) * (ny + 2) * (nz + 2);
    if (bytes_overlap(partials, pb, dw, 4ll * kTaps * kC * kC) || bytes_overlap(partials, pb, db, 4ll * kC) ||
        bytes_overlap(partials, pb, dz, 4 * vox * kC) || bytes_overlap(partials, pb, x, 2 * pvox * kC))
        return RTM_EALIAS;
    const Vol v{nx, ny, nz};
    CNN_CHECK_DEVICE();
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz);
    hipLaunchKernelGGL(k_conv3d_wgrad<true>, grid, dim3(256), 0, stream, v, x, dz, dw, db, partials);
    int st = status();
    if (st != RTM_OK) return st;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((kWgradSlot + 63) / 64), dim3(64 * kReduceGroups), 0, stream, partials,
                       (long long)grid.x * grid.y * grid.z, dw, db);
    return status();
}

int rtm_cnn_relu_backward(int32_t nx, int32_t ny, int32_t nz, const float *y, const float *dy, int32_t relu,
                          int32_t channels, float *dz32, uint16_t *dz16, hipStream_t stream)
{
    if (!vol_ok(nx, ny, nz) || !dy || !dz32 || !dz16 || (relu && !y) || channels < 0 || channels > kC)
        return RTM_EINVAL;
    const Vol v{nx, ny, nz};
    const long long n = (long long)nx * ny * nz * kC;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_relu_backward, dim3(nblk(n)), dim3(256), 0, stream, v, y, dy, (int)relu, (int)channels, dz32,
                       dz16);
    return status();
}

int rtm_cnn_loss_grad(int32_t nx, int32_t ny, int32_t nz, const float *out, const float *target, int32_t channels,
                      float weight, const float *mask, float *dz32, uint16_t *dz16, double *loss, hipStream_t stream)
{
    if (!vol_ok(nx, ny, nz) || !out || !target || !dz32 || !dz16 || channels < 0 || channels > kC || !(weight >= 0.0f))
        return RTM_EINVAL;
    const Vol v{nx, ny, nz};
    const long long n = (long long)nx * ny * nz * kC;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_loss_grad, dim3(nblk(n)), dim3(256), 0, stream, v, out, target, (int)channels, weight, mask,
                       dz32, dz16, loss);
    return status();
}

int rtm_cnn_weight_flip(const uint16_t *w, uint16_t *wt, hipStream_t stream)
{
    if (!w || !wt || w == wt) return RTM_EINVAL;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_weight_flip, dim3(nblk(kTaps * kC * kC)), dim3(256), 0, stream, w, wt);
    return status();
}

int rtm_cnn_adam(float *param, const float *grad, float *m1, float *m2, int32_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, uint16_t *param_bf16, hipStream_t stream)
{
    if (!param || !grad || !m1 || !m2 || n < 0 || step < 1) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    const float c1 = 1.0f - (float)__builtin_pow(beta1, step), c2 = 1.0f - (float)__builtin_pow(beta2, step);
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, stream, param, grad, m1, m2, (int)n, lr, beta1, beta2, eps,
                       c1, c2, param_bf16);
    return status();
}

int rtm_cnn_to_bf16(const float *a, uint16_t *b, int32_t n, hipStream_t stream)
{
    if (!a || !b || n < 0) return RTM_EINVAL;
    if (n == 0) return RTM_OK;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, stream, a, b, (int)n);
    return status();
}

int rtm_cnn_pack_input(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *velocity,
                       float v_ref, float v_scale, const float *scale, const float *noise, uint16_t *x,
                       hipStream_t stream)
{
    if (!grid_ok(grid) || !u_cur || !u_prv || !velocity || !scale || !x || !(v_scale > 0.0f)) return RTM_EINVAL;
    if (!vol_ok(grid->nx, grid->ny, grid->nz)) return RTM_EINVAL;
    const G g = make_g(grid);
    const Vol v{grid->nx, grid->ny, grid->nz};
    const long long n = (long long)g.nx * g.ny * g.nz;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(n)), dim3(256), 0, stream, g, v, u_cur, u_prv, velocity, v_ref,
                       1.0f / v_scale, scale, noise, x);
    return status();
}

int rtm_cnn_apply_correction(const rtm_grid *grid, float *u_cur, float *u_prv, const float *out, int32_t out_channels,
                             const float *mask, const float *scale, hipStream_t stream)
{
    if (!grid_ok(grid) || !u_cur || !u_prv || !out || !scale || u_cur == u_prv || out_channels < 2 ||
        out_channels > kC)
        return RTM_EINVAL;
    const G g = make_g(grid);
    const long long n = (long long)g.nx * g.ny * g.nz;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_apply_correction, dim3(nblk(n)), dim3(256), 0, stream, g, u_cur, u_prv, out,
                       (int)out_channels, mask, scale);
    return status();
}

int rtm_cnn_target(const rtm_grid *grid, const float *ref_cur, const float *ref_prv, const float *u_cur,
                   const float *u_prv, const float *scale, const float *noise, float *target, hipStream_t stream)
{
    if (!grid_ok(grid) || !ref_cur || !ref_prv || !u_cur || !u_prv || !scale || !target) return RTM_EINVAL;
    const G g = make_g(grid);
    const long long n = (long long)g.nx * g.ny * g.nz;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_target, dim3(nblk(n)), dim3(256), 0, stream, g, ref_cur, ref_prv, u_cur, u_prv, scale, noise,
                       target);
    return status();
}

int rtm_restrict(const rtm_grid *fine, const rtm_grid *coarse, const float *u_fine, float *u_coarse, int32_t mode,
                 hipStream_t stream)
{
    if (!grid_ok(fine) || !grid_ok(coarse) || !u_fine || !u_coarse) return RTM_EINVAL;
    if (mode != RTM_RESTRICT_INJECT && mode != RTM_RESTRICT_FULL) return RTM_EINVAL;
    // fine (2i, 2j, 2k) must be owned for every coarse cell (full weighting then reads at most one
    // ghost layer, which exists since the radius is >= 2)
    if (2 * (coarse->nx - 1) >= fine->nx || 2 * (coarse->ny - 1) >= fine->ny || 2 * (coarse->nz - 1) >= fine->nz)
        return RTM_EINVAL;
    const G f = make_g(fine), c = make_g(coarse);
    const long long n = (long long)c.nx * c.ny * c.nz;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_restrict, dim3(nblk(n)), dim3(256), 0, stream, f, c, u_fine, u_coarse,
                       (int)(mode == RTM_RESTRICT_FULL));
    return status();
}

int rtm_prolong(const rtm_grid *coarse, const rtm_grid *fine, const float *u_coarse, float *u_fine, hipStream_t stream)
{
    if (!grid_ok(fine) || !grid_ok(coarse) || !u_fine || !u_coarse) return RTM_EINVAL;
    // every fine cell's coarse neighbours are owned or in the first ghost layer
    if (fine->nx > 2 * coarse->nx || fine->ny > 2 * coarse->ny || fine->nz > 2 * coarse->nz) return RTM_EINVAL;
    const G f = make_g(fine), c = make_g(coarse);
    const long long n = (long long)f.nx * f.ny * f.nz;
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_prolong, dim3(nblk(n)), dim3(256), 0, stream, c, f, u_coarse, u_fine);
    return status();
}

int rtm_field_absmax(const rtm_grid *grid, const float *u, float *out, hipStream_t stream)
{
    if (!grid_ok(grid) || !u || !out) return RTM_EINVAL;
    const G g = make_g(grid);
    CNN_CHECK_DEVICE();
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, stream, out);
    int st = status();
    if (st != RTM_OK) return st;
    const long long n = (long long)g.nx * g.ny * g.nz;
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((n + 1023) / 1024, 4096));
    if (n + 4LL * 256 * blocks < (1LL << 31))
        hipLaunchKernelGGL(k_absmax_cells<int>, dim3(blocks), dim3(256), 0, stream, g, u, out);
    else
        hipLaunchKernelGGL(k_absmax_cells<long long>, dim3(blocks), dim3(256), 0, stream, g, u, out);
    return status();
}

}  // extern "C"
