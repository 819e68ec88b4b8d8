// merf_render.hip -- gfx950 kernels of the MERF deferred volume renderer.
//
// One wave64 renders an 8x8 tile of pixels, one ray per lane, so the rays of
// a wave are coherent and their plane and grid gathers fall on nearby texels.
// Per lane (MERF, arXiv 2302.12249):
//   1. pinhole ray (o, d);
//   2. the ray is cut at the parameters where the region of the
//      piecewise-projective contraction changes (Sec. 4.2, Eq. 7); each piece
//      maps to a straight contracted segment, handled one at a time;
//   3. each segment is marched on a uniform lattice of contracted step s
//      (sample at each interval midpoint, last interval shortened); a sample
//      is evaluated only if every occupancy level marks its cell occupied
//      (Sec. 6); in empty space the march jumps to the first lattice sample
//      past the exit of an empty box (ray-box slab test in contracted space,
//      exact because the segment is straight): by default the largest empty
//      cube ahead, from a grid derived from the levels at upload, otherwise
//      the empty cell of the first empty level;
//   4. evaluated samples are parked in LDS; the wave shades up to 64 parked
//      samples at once, whoever's they are: gather the 3D grid (trilinear,
//      one brick per sample thanks to the apron) and the three planes
//      (bilinear), dequantise (Eq. 8; the fp32 path applies it to the
//      interpolated codes, the same value up to rounding), sum (Eq. 5),
//      decode (Eq. 6) -- density first, appearance only when alpha != 0;
//      each lane then composites its own samples in ray order (Eq. 1-2);
//   5. marching stops when the transmittance drops below t_min (Sec. 6);
//   6. the deferred MLP h(C_d, F, d) runs once per pixel (Eq. 3, App. B).
// Before a launch, a prepass (k_tile_cost, k_tile_order) marches a few
// probe rays per tile and orders the tiles by their estimated work, heaviest
// first; the served kernel (k_render_served) runs the same per-tile code on
// requests of several scenes described in device memory.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "merf_device.h"

namespace merf {

namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr float kRcp255 = 1.0f / 255.0f;
// Samples are never skipped past a cell exit by more than this (contracted
// units): FP32 error of the exit parameter is below 1e-6.
constexpr float kSkipGuard = 2e-6f;

// ---------------------------------------------------------------------------
// Eq. 8: code b -> 2 m b / 255 - m, correctly rounded to float32.
// k = m (2b - 255) is an exact small integer; q = k * RN(1/255) is then
// corrected by one residual step (Markstein), which gives the correctly
// rounded quotient k / 255 for every code and m in {7, 14} (checked
// exhaustively by the test-suite).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float deq_f32(uint32_t b, float m2, float m255) {
    float k = fmaf((float)b, m2, -m255);
    float q = k * kRcp255;
    float r = fmaf(-q, 255.0f, k);
    return fmaf(r, kRcp255, q);
}


__device__ __forceinline__ uint32_t byte_of(uint32_t w, int i) { return (w >> (8 * i)) & 0xffu; }

// Two codes as the float16 subnormals b * 2^-24, which are exact: mixed-
// precision FMAs (v_fma_mix_f32) then take them as operands directly, so an
// interpolation term costs one instruction instead of a convert and an FMA.
// The sums come out scaled by 2^-24 exactly (a power of two, far from the
// float32 range limits), which the Eq. 8 scale absorbs.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f16x2 as_f16x2(uint32_t w) { return __builtin_bit_cast(f16x2, w); }
// bytes 0 and 2 of w
__device__ __forceinline__ f16x2 codes02(uint32_t w) { return as_f16x2(w & 0x00ff00ffu); }
// bytes 1 and 3 of w
__device__ __forceinline__ f16x2 codes13(uint32_t w) { return as_f16x2(__builtin_amdgcn_perm(0u, w, 0x0c030c01u)); }
// byte 0 of a and byte 0 of b
__device__ __forceinline__ f16x2 codes0_0(uint32_t a, uint32_t b) {
    return as_f16x2(__builtin_amdgcn_perm(b, a, 0x0c040c00u));
}

// byte j of a and byte j of b
template <int j>
__device__ __forceinline__ f16x2 codes_jj(uint32_t a, uint32_t b) {
    return as_f16x2(__builtin_amdgcn_perm(b, a, 0x0c000c00u | ((4u + j) << 16) | (uint32_t)j));
}

// Eq. 8 to float16 of a code given as the subnormal b 2^-24, with
// a24 = 2^24 RN32(2m/255) (the scale the upload computes, times 2^24): the
// product is b RN32(2m/255) exactly, so this is RN16(RN32(b a - m)), which
// equals the correctly rounded float16 of the exact 2mb/255 - m for every
// code and m in {7, 14} (checked exhaustively on the host, and bit for bit on
// the device through merf_dequantize, which runs this routine).  Returned
// widened to float; the compiler fuses the FMA and the rounding to float16
// into one mixed-precision instruction.
__device__ __forceinline__ float deq_f16(_Float16 code, float a24, float m) {
    return (float)(_Float16)fmaf((float)code, a24, -m);
}

// Hardware reciprocal (v_rcp_f32, 1 ulp); rcp(+-0) = +-inf.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Eq. 7 regions: 0 = unit cube, 1 + 2j + (x_j < 0) = outer region of axis j.
// Ties pick the first axis.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int region_of(float x, float y, float z) {
    float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int j = 0;
    float r = ax, v = x;
    if (ay > r) { r = ay; j = 1; v = y; }
    if (az > r) { r = az; j = 2; v = z; }
    if (r <= 1.0f) return 0;
    return 1 + 2 * j + (v < 0.0f ? 1 : 0);
}

// Projective map of region reg (Eq. 7): y_j = (2 - 1/|x_j|) s, y_k = x_k/|x_j|.
__device__ __forceinline__ float3 map_region(int reg, float3 x) {
    if (reg == 0) return x;
    int j = (reg - 1) >> 1;
    float s = ((reg - 1) & 1) ? -1.0f : 1.0f;
    float xj = j == 0 ? x.x : (j == 1 ? x.y : x.z);
    float ia = rcp(fabsf(xj));
    float3 y = make_float3(x.x * ia, x.y * ia, x.z * ia);
    float yj = (2.0f - ia) * s;
    if (j == 0) y.x = yj; else if (j == 1) y.y = yj; else y.z = yj;
    return y;
}

// Contracted image of the ray's point at infinity in region reg.
__device__ __forceinline__ float3 limit_point(int reg, float3 d) {
    int j = (reg - 1) >> 1;
    float s = ((reg - 1) & 1) ? -1.0f : 1.0f;
    float dj = j == 0 ? d.x : (j == 1 ? d.y : d.z);
    float ia = rcp(fabsf(dj));
    float3 y = make_float3(d.x * ia, d.y * ia, d.z * ia);
    if (j == 0) y.x = 2.0f * s; else if (j == 1) y.y = 2.0f * s; else y.z = 2.0f * s;
    return y;
}

// Preimage of a contracted point in region reg (world-length deltas).
__device__ __forceinline__ float3 unmap_region(int reg, float3 y) {
    if (reg == 0) return y;
    int j = (reg - 1) >> 1;
    float s = ((reg - 1) & 1) ? -1.0f : 1.0f;
    float yj = j == 0 ? y.x : (j == 1 ? y.y : y.z);
    float a = rcp(2.0f - s * yj);
    float3 x = make_float3(y.x * a, y.y * a, y.z * a);
    if (j == 0) x.x = s * a; else if (j == 1) x.y = s * a; else x.z = s * a;
    return x;
}

struct Candidates {
    float c[12];
};

__device__ __forceinline__ float valid_t(float t) { return (t > 0.0f && t < kInf) ? t : kInf; }

// Parameters t > 0 where the ray can change region: x_j = +-1, x_j = +-x_k.
// Hardware reciprocals (1 ulp) replace divisions: a breakpoint is only needed
// to FP32 accuracy, and a zero denominator still gives +-inf (no candidate).
__device__ __forceinline__ Candidates make_candidates(float3 o, float3 d) {
    Candidates C;
    const float ix = rcp(d.x), iy = rcp(d.y), iz = rcp(d.z);
    C.c[0] = valid_t((1.0f - o.x) * ix);
    C.c[1] = valid_t((-1.0f - o.x) * ix);
    C.c[2] = valid_t((1.0f - o.y) * iy);
    C.c[3] = valid_t((-1.0f - o.y) * iy);
    C.c[4] = valid_t((1.0f - o.z) * iz);
    C.c[5] = valid_t((-1.0f - o.z) * iz);
    C.c[6] = valid_t((o.y - o.x) * rcp(d.x - d.y));
    C.c[7] = valid_t((-o.y - o.x) * rcp(d.x + d.y));
    C.c[8] = valid_t((o.z - o.x) * rcp(d.x - d.z));
    C.c[9] = valid_t((-o.z - o.x) * rcp(d.x + d.z));
    C.c[10] = valid_t((o.z - o.y) * rcp(d.y - d.z));
    C.c[11] = valid_t((-o.z - o.y) * rcp(d.y + d.z));
    return C;
}

// Smallest of n candidates strictly greater than t (kInf if none): each
// candidate is masked to kInf unless above t, then three-way minima.
template <int n>
__device__ __forceinline__ float next_of(const float *c, float t) {
    float m = kInf;
#pragma unroll
    for (int i = 0; i < n; i += 3) {
        const float a = c[i] > t ? c[i] : kInf;
        const float b = i + 1 < n && c[i + 1] > t ? c[i + 1] : kInf;
        const float e = i + 2 < n && c[i + 2] > t ? c[i + 2] : kInf;
        m = fminf(m, fminf(a, fminf(b, e)));
    }
    return m;
}
__device__ __forceinline__ float next_candidate(const Candidates &C, float t) { return next_of<12>(C.c, t); }

__device__ __forceinline__ int region_at(float3 o, float3 d, float t) {
    return region_of(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
}

// 24-bit multiply (v_mul_u32_u24, full rate; a 32-bit integer multiply is
// quarter rate): both factors below 2^24, the low 32 bits of the product.
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return __umul24(a, b); }

// Cell of a grid of r cells a side at scaled coordinate v = (p + 2) r / 4,
// clamped to [0, r - 1] on both sides (one median instruction), so that a
// lookup stays inside the grid whatever the point.
__device__ __forceinline__ int cell_index(float v, int r) { return max(min((int)v, r - 1), 0); }

// Byte offset of cell (x, y, z) of an r^3 z-major grid; every factor is
// below 2^24 (r <= 1024).
__device__ __forceinline__ uint32_t cell_offset(int x, int y, int z, int r) {
    return mul24((uint32_t)z, mul24((uint32_t)r, (uint32_t)r)) + mul24((uint32_t)y, (uint32_t)r) + (uint32_t)x;
}

// Number of lanes below this one whose bit is set in the wave mask m.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ float sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// XCD-aware tile order.  Consecutive workgroups are dispatched round-robin
// over the 8 XCDs (workgroup b runs on XCD b % 8 as that XCD's (b / 8)-th),
// with no balancing between XCDs.  Each XCD therefore gets runs of
// kXcdChunk consecutive tiles (neighbouring tiles gather neighbouring texels
// and share that XCD's L2), and the runs are dealt to the XCDs in turn over
// the whole launch, so every XCD gets a similar share of the image's work.
// Workgroups past the last whole round of runs keep their own tile.
constexpr int kXcdChunk = 4;
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    constexpr int nx = 8;
    const int full = n / (nx * kXcdChunk) * (nx * kXcdChunk);
    if (bid >= full) return bid;
    const int x = bid % nx, i = bid / nx;
    return ((i / kXcdChunk) * nx + x) * kXcdChunk + i % kXcdChunk;
}

struct Accum {
    float T, cd0, cd1, cd2, f0, f1, f2, f3;
};

struct Counters {
    uint32_t occ_lookups, visited, evaluated, contributing, opens;
};

// Phase profile of the statistics variant (RenderBatch::phases): shader-clock
// timestamps taken at points every lane of the wave passes together, so each
// interval is wave time, added to the phase it belongs to.  Lane i keeps the
// sum of slot i (one register for all slots; a wave's sums stay below 2^32).
template <bool kOn>
struct PhaseClock {
    uint32_t t = 0, v = 0;          // low word of the last timestamp; this lane's sum
    __device__ __forceinline__ void start() {
        if (kOn) t = (uint32_t)__builtin_amdgcn_s_memtime();
    }
    __device__ __forceinline__ void count(int slot, uint32_t x = 1) {
        if (kOn) v += (int)threadIdx.x == slot ? x : 0u;
    }
    __device__ __forceinline__ void lap(int slot) {
        if (kOn) {
            const uint32_t n = (uint32_t)__builtin_amdgcn_s_memtime();
            count(slot, n - t);     // modulo 2^32: intervals are far shorter
            t = n;
        }
    }
};

template <typename T>
__device__ __forceinline__ T load_at(const uint8_t *base, uint32_t off) {
    return *reinterpret_cast<const T *>(base + off);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load: two adjacent 8-byte texels.
__device__ __forceinline__ u32x4 load_pair(const uint8_t *base, uint32_t off) {
    return *reinterpret_cast<const u32x4 *>(base + off);
}

// Byte offsets of the 20 texels one sample reads.  Planes: the (u, v) and
// (u + 1, v) texels of row v start at op[p] and those of row v + 1 at
// op[p] + prow.  Grid: the 2x2x2 footprint of brick slot brick_index[bi]
// starts at byte ol of that brick.
struct Footprint {
    uint32_t op[3], prow, bi, ol;
    float ex, ey, ez;   // plane texel fractions
    float fx, fy, fz;   // grid voxel fractions
};

// Scene accessors take the scene as S = const DevScene (a kernel argument)
// or as a constant-address-space DevScene (a slot of a served launch's
// table), so both read it with scalar loads that may be repeated at will.
template <typename S>
__device__ __forceinline__ Footprint footprint(const S &sc, float3 p) {
    Footprint f;
    // ---- three planes, bilinear: P_x(y, z), P_y(x, z), P_z(x, y)
    const float ps = sc.p_scale, ps2 = sc.p_off, pmax = sc.p_max;
    float hx = __builtin_amdgcn_fmed3f(fmaf(p.x, ps, ps2), 0.0f, pmax);
    float hy = __builtin_amdgcn_fmed3f(fmaf(p.y, ps, ps2), 0.0f, pmax);
    float hz = __builtin_amdgcn_fmed3f(fmaf(p.z, ps, ps2), 0.0f, pmax);
    int jx = min((int)hx, sc.R - 2), jy = min((int)hy, sc.R - 2), jz = min((int)hz, sc.R - 2);
    f.ex = hx - (float)jx; f.ey = hy - (float)jy; f.ez = hz - (float)jz;
    const uint32_t row = (uint32_t)sc.R * kChannels, plane = (uint32_t)sc.R * row;
    f.prow = row;
    // (R <= 8192: texel indices and the row of 8 R bytes are below 2^24, and
    // every offset below 2^31)
    f.op[0] = mul24((uint32_t)jz, row) + (uint32_t)jy * kChannels;
    f.op[1] = plane + mul24((uint32_t)jz, row) + (uint32_t)jx * kChannels;
    f.op[2] = 2u * plane + mul24((uint32_t)jy, row) + (uint32_t)jx * kChannels;
    // ---- sparse 3D grid, trilinear inside one apron brick
    const float gs = sc.g_scale, gs2 = sc.g_off, gmax = sc.g_max;
    float gx = __builtin_amdgcn_fmed3f(fmaf(p.x, gs, gs2), 0.0f, gmax);
    float gy = __builtin_amdgcn_fmed3f(fmaf(p.y, gs, gs2), 0.0f, gmax);
    float gz = __builtin_amdgcn_fmed3f(fmaf(p.z, gs, gs2), 0.0f, gmax);
    int ix = min((int)gx, sc.L - 2), iy = min((int)gy, sc.L - 2), iz = min((int)gz, sc.L - 2);
    f.fx = gx - (float)ix; f.fy = gy - (float)iy; f.fz = gz - (float)iz;
    f.bi = mul24((uint32_t)(iz >> 3), mul24((uint32_t)sc.nbl, (uint32_t)sc.nbl)) +
           mul24((uint32_t)(iy >> 3), (uint32_t)sc.nbl) + (uint32_t)(ix >> 3);
    f.ol = (uint32_t)((((iz & 7) * kBrick + (iy & 7)) * kBrick + (ix & 7)) * kChannels);
    return f;
}

// The ten 16-byte texel pairs of a sample: 6 plane pairs, 4 grid pairs.
struct Texels {
    u32x4 t[6], g[4];
};

// Issue every load of a sample before waiting on any: the brick index first
// (the brick loads depend on it), then the plane pairs, which overlap its
// round trip, then the brick pairs.  The empty asm takes all ten vectors, so
// the compiler neither splits them into per-word loads nor sinks any behind
// the alpha test, and places one wait before it.  Every array is present on
// the device (a scene without a grid or without planes reads an all-zero
// stand-in), so nothing here branches.
template <typename S>
__device__ __forceinline__ Texels gather(const S &sc, const Footprint &f) {
    Texels x;
    const int brick = load_at<int>(reinterpret_cast<const uint8_t *>(sc.brick_index), f.bi * 4u);
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
        x.t[2 * pl] = load_pair(sc.planes, f.op[pl]);
        x.t[2 * pl + 1] = load_pair(sc.planes, f.op[pl] + f.prow);
    }
    constexpr uint32_t sy = kBrick * kChannels, sz = kBrick * kBrick * kChannels;
    // (fewer than 2^31 / kBrickBytes bricks: the upload checks it)
    const uint32_t ob = mul24((uint32_t)brick, kBrickBytes) + f.ol;
    x.g[0] = load_pair(sc.bricks, ob);
    x.g[1] = load_pair(sc.bricks, ob + sy);
    x.g[2] = load_pair(sc.bricks, ob + sz);
    x.g[3] = load_pair(sc.bricks, ob + sz + sy);
    asm volatile("" : "+v"(x.t[0]), "+v"(x.t[1]), "+v"(x.t[2]), "+v"(x.t[3]), "+v"(x.t[4]), "+v"(x.t[5]),
                 "+v"(x.g[0]), "+v"(x.g[1]), "+v"(x.g[2]), "+v"(x.g[3]));
    return x;
}

// Shaded sample: 1 - alpha and, when alpha != 0, the sigmoids of the diffuse
// colour and the features (Eq. 6).
struct SampleResult {
    float trans;
    float sg[7];
};

// One evaluated sample: gather, dequantise, decode.
// All offsets are 32-bit (the upload keeps every array below 2 GiB) and are
// added to uniform base pointers, so no 64-bit address arithmetic runs per lane.
template <int kFeat, typename S>
__device__ __forceinline__ SampleResult eval_sample(const S &sc, float3 p, float delta) {
    const Footprint f = footprint(sc, p);
    const Texels x = gather(sc, f);
    // texel words of the 20 texels (lo = channels 0..3, hi = 4..7) and their
    // weights: 8 grid corners, then 4 texels of each plane.  An absent source
    // reads zero codes, so its weights do not matter.
    uint32_t lo[20], hi[20];
    float w[20];
    {
        const float fu[3] = {f.ey, f.ex, f.ex}, fv[3] = {f.ez, f.ez, f.ey};   // (u, v) = (y, z), (x, z), (x, y)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
            const float au = 1.0f - fu[pl], av = 1.0f - fv[pl];
            const u32x4 r0 = x.t[2 * pl], r1 = x.t[2 * pl + 1];
            lo[8 + 4 * pl] = r0.x; hi[8 + 4 * pl] = r0.y; w[8 + 4 * pl] = au * av;
            lo[9 + 4 * pl] = r0.z; hi[9 + 4 * pl] = r0.w; w[9 + 4 * pl] = fu[pl] * av;
            lo[10 + 4 * pl] = r1.x; hi[10 + 4 * pl] = r1.y; w[10 + 4 * pl] = au * fv[pl];
            lo[11 + 4 * pl] = r1.z; hi[11 + 4 * pl] = r1.w; w[11 + 4 * pl] = fu[pl] * fv[pl];
        }
        // corners (x, x + 1) at (y, z), (y + 1, z), (y, z + 1), (y + 1, z + 1)
        const float ax = 1.0f - f.fx, ay = 1.0f - f.fy, az = 1.0f - f.fz;
        const float wyz[4] = {ay * az, f.fy * az, ay * f.fz, f.fy * f.fz};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            lo[2 * i] = x.g[i].x; hi[2 * i] = x.g[i].y; w[2 * i] = ax * wyz[i];
            lo[2 * i + 1] = x.g[i].z; hi[2 * i + 1] = x.g[i].w; w[2 * i + 1] = f.fx * wyz[i];
        }
    }
    // ---- Eq. 8 dequantises each code affinely, q(b) = a b - m with a = 2m/255,
    // and the weights of each present source sum to one, so
    // sum_i w_i q(b_i) = a * sum_i w_i b_i - n m exactly (n sources: 4 for
    // grid + planes).  The FP32 path
    // (kFeat = 0) interpolates the codes and applies the affine map
    // once per channel: the same real number with one convert and one FMA per
    // texel and channel; the two FP32 evaluations differ by rounding only
    // (below 1e-6 relative).  The exact-FP16 path (kFeat = 1) dequantises
    // every code to its correctly rounded float16 value first (deq_f16) and
    // interpolates those values with FP32 weights and FP32 sums.  The
    // FP16-interpolation path (kFeat = 2) computes density as the FP32 path
    // does and interpolates the appearance channels from float16 operands:
    // the weights rounded to float16, the codes exact, each pair of texels
    // summed by one dot product with FP32 accumulation (v_dot2_f32_f16).
    // (a = d_scale or f_scale, n m = -d_off or -f_off, precomputed)
    const float md = sc.m_density, mf = sc.m_feature;
    // ---- density first (Sec. 6): appearance is read only when alpha != 0
    float s0 = 0.0f;
    if constexpr (kFeat == 1) {
        // a stand-in source (scene without grid or without planes) reads code
        // 0, whose float16 value is -m: its texels get weight 0 here, so that
        // the sum holds the present sources only (Eq. 5)
#pragma unroll
        for (int i = 0; i < 20; ++i) w[i] *= i < 8 ? sc.grid_w : sc.planes_w;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const f16x2 c = codes0_0(lo[2 * k], lo[2 * k + 1]);
            s0 = fmaf(w[2 * k], deq_f16(c.x, sc.d_scale24, md), s0);
            s0 = fmaf(w[2 * k + 1], deq_f16(c.y, sc.d_scale24, md), s0);
        }
    } else {
        // texel pairs: the density codes of texels 2k and 2k + 1 in one word
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const f16x2 c = codes0_0(lo[2 * k], lo[2 * k + 1]);
            s0 = fmaf(w[2 * k], (float)c.x, s0);
            s0 = fmaf(w[2 * k + 1], (float)c.y, s0);
        }
        s0 = fmaf(s0, sc.d_scale24, sc.d_off);
    }
    SampleResult r;
    float tau = __expf(s0);                       // Eq. 6
    r.trans = __expf(-tau * delta);               // e^{-tau delta} = 1 - alpha (Eq. 1)
    if (1.0f - r.trans > 0.0f) {
        float sa[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) sa[c] = 0.0f;
        if constexpr (kFeat == 2) {
            // texel pairs (2k, 2k + 1): their weights and the codes of one
            // channel in one register each
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const f16x2 wk = {(_Float16)w[2 * k], (_Float16)w[2 * k + 1]};
                const uint32_t la = lo[2 * k], lb = lo[2 * k + 1], ha = hi[2 * k], hb = hi[2 * k + 1];
                sa[0] = __builtin_amdgcn_fdot2(wk, codes_jj<1>(la, lb), sa[0], false);
                sa[1] = __builtin_amdgcn_fdot2(wk, codes_jj<2>(la, lb), sa[1], false);
                sa[2] = __builtin_amdgcn_fdot2(wk, codes_jj<3>(la, lb), sa[2], false);
                sa[3] = __builtin_amdgcn_fdot2(wk, codes_jj<0>(ha, hb), sa[3], false);
                sa[4] = __builtin_amdgcn_fdot2(wk, codes_jj<1>(ha, hb), sa[4], false);
                sa[5] = __builtin_amdgcn_fdot2(wk, codes_jj<2>(ha, hb), sa[5], false);
                sa[6] = __builtin_amdgcn_fdot2(wk, codes_jj<3>(ha, hb), sa[6], false);
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) sa[c] = fmaf(sa[c], sc.f_scale24, sc.f_off);
        } else if constexpr (kFeat == 1) {
            const float af = sc.f_scale24;
#pragma unroll
            for (int i = 0; i < 20; ++i) {
                const f16x2 l02 = codes02(lo[i]), l13 = codes13(lo[i]);
                const f16x2 h02 = codes02(hi[i]), h13 = codes13(hi[i]);
                sa[0] = fmaf(w[i], deq_f16(l13.x, af, mf), sa[0]);
                sa[1] = fmaf(w[i], deq_f16(l02.y, af, mf), sa[1]);
                sa[2] = fmaf(w[i], deq_f16(l13.y, af, mf), sa[2]);
                sa[3] = fmaf(w[i], deq_f16(h02.x, af, mf), sa[3]);
                sa[4] = fmaf(w[i], deq_f16(h13.x, af, mf), sa[4]);
                sa[5] = fmaf(w[i], deq_f16(h02.y, af, mf), sa[5]);
                sa[6] = fmaf(w[i], deq_f16(h13.y, af, mf), sa[6]);
            }
        } else {
            // per texel pair: channel 2 of both texels from one permute, so
            // 7 permutes or masks extract the 14 codes of the pair
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const f16x2 c2 = codes_jj<2>(lo[2 * k], lo[2 * k + 1]);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int i = 2 * k + t;
                    const f16x2 l13 = codes13(lo[i]);
                    const f16x2 h02 = codes02(hi[i]), h13 = codes13(hi[i]);
                    sa[0] = fmaf(w[i], (float)l13.x, sa[0]);
                    sa[1] = fmaf(w[i], (float)(t ? c2.y : c2.x), sa[1]);
                    sa[2] = fmaf(w[i], (float)l13.y, sa[2]);
                    sa[3] = fmaf(w[i], (float)h02.x, sa[3]);
                    sa[4] = fmaf(w[i], (float)h13.x, sa[4]);
                    sa[5] = fmaf(w[i], (float)h02.y, sa[5]);
                    sa[6] = fmaf(w[i], (float)h13.y, sa[6]);
                }
            }
#pragma unroll
            for (int c = 0; c < 7; ++c) sa[c] = fmaf(sa[c], sc.f_scale24, sc.f_off);
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) r.sg[c] = sigmoid(sa[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) r.sg[c] = 0.0f;
    }
    return r;
}

// Front-to-back compositing of one shaded sample (Eq. 1-2).
template <bool kStats>
__device__ __forceinline__ void composite(Accum &acc, const SampleResult &r, Counters &cnt) {
    const float alpha = 1.0f - r.trans;
    if (kStats) ++cnt.evaluated;
    if (alpha > 0.0f) {
        if (kStats) ++cnt.contributing;
        const float wt = acc.T * alpha;
        acc.cd0 = fmaf(wt, r.sg[0], acc.cd0);
        acc.cd1 = fmaf(wt, r.sg[1], acc.cd1);
        acc.cd2 = fmaf(wt, r.sg[2], acc.cd2);
        acc.f0 = fmaf(wt, r.sg[3], acc.f0);
        acc.f1 = fmaf(wt, r.sg[4], acc.f1);
        acc.f2 = fmaf(wt, r.sg[5], acc.f2);
        acc.f3 = fmaf(wt, r.sg[6], acc.f3);
        acc.T *= r.trans;
    }
}

// March state of one straight contracted segment A -> B (region reg) that
// covers the world parameters [ta, tb] of the ray (B itself is recomputed by
// segment_end where needed).
struct Segment {
    float3 A, e;                    // contracted start, unit direction
    float len, iex, iey, iez;       // length; inverse direction (+-inf where e = +-0)
    float tb;                       // world parameter of the end (kInf: last)
    int n, k, reg, reg_next;        // interval count, next interval, regions
    uint32_t doff;                  // byte offset of the empty-space grid of this direction's octant
};

// Contracted end point of the segment of region reg that ends at world
// parameter tb (kInf: the limit point of the ray).
__device__ __forceinline__ float3 segment_end(float3 o, float3 d, float tb, int reg) {
    return tb < kInf ? map_region(reg, make_float3(fmaf(tb, d.x, o.x), fmaf(tb, d.y, o.y), fmaf(tb, d.z, o.z)))
                     : limit_point(reg, d);
}

// Set up the segment of the ray that starts at world parameter ta in region
// reg: find where the region changes (Eq. 7 breakpoints), map both ends.
// Every region is convex, so the ray leaves reg at the first breakpoint after
// ta on one of reg's own boundary planes that it crosses outward: inside the
// cube any face x_j = +-1; in the outer region of axis a (sign s) its face
// x_a = s when |x_a| shrinks, and a plane x_a = +-x_k when |x_k| grows past
// |x_a| there.  The direction of a crossing follows from the signs of the
// direction's components, so it is exact even where several planes meet
// (a ray through a cube edge crosses the seam between two outer regions into
// the region it enters, not out of it).  The region entered is read at the
// midpoint to the next breakpoint of the full set; where that midpoint is
// within rounding of the exit and still reads reg, it is the region across
// the exit plane (the outer region of face x_j = +-1, the cube across a face
// x_a = s, axis k with the sign x_k takes across x_a = +-x_k).
__device__ __forceinline__ void open_segment(float3 o, float3 d, float ta, int reg, float istep, uint32_t oct_stride,
                                             Segment &s) {
    const Candidates C = make_candidates(o, d);
    // the six boundary planes of reg: cube {0..5}; axis 0 {0, 1, 6, 7, 8, 9};
    // axis 1 {2, 3, 6, 7, 10, 11}; axis 2 {4, 5, 8, 9, 10, 11}
    const int ax = (reg - 1) >> 1, neg = (reg - 1) & 1;
    const bool in_cube = reg == 0, a0 = !in_cube && ax == 0, a1 = !in_cube && ax == 1;
    float cr[6];
    cr[0] = in_cube || a0 ? C.c[0] : (a1 ? C.c[2] : C.c[4]);
    cr[1] = in_cube || a0 ? C.c[1] : (a1 ? C.c[3] : C.c[5]);
    cr[2] = in_cube ? C.c[2] : (a0 || a1 ? C.c[6] : C.c[8]);
    cr[3] = in_cube ? C.c[3] : (a0 || a1 ? C.c[7] : C.c[9]);
    cr[4] = in_cube ? C.c[4] : (a0 ? C.c[8] : C.c[10]);
    cr[5] = in_cube ? C.c[5] : (a0 ? C.c[9] : C.c[11]);
    // outer regions: the other axes k1 < k2, and for each plane whether
    // crossing it leaves the region (|x_a| shrinks below 1, or |x_k| grows
    // past |x_a|)
    const int k1 = a0 ? 1 : 0, k2 = ax == 2 ? 1 : 2;
    const float da = ax == 0 ? d.x : (ax == 1 ? d.y : d.z);
    const float dk1 = k1 == 0 ? d.x : d.y, dk2 = k2 == 1 ? d.y : d.z;
    const bool sneg = neg != 0;
    bool out[6];
    out[0] = in_cube || (!sneg && da < 0.0f);
    out[1] = in_cube || (sneg && da > 0.0f);
    out[2] = in_cube || ((dk1 > da) != sneg);
    out[3] = in_cube || ((da + dk1 < 0.0f) != sneg);
    out[4] = in_cube || ((dk2 > da) != sneg);
    out[5] = in_cube || ((da + dk2 < 0.0f) != sneg);
    float tb = kInf;
    int hit = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const bool nearer = out[i] && cr[i] > ta && cr[i] < tb;    // ties: the first plane
        tb = nearer ? cr[i] : tb;
        hit = nearer ? i : hit;
    }
    // the region across the exit plane (regions are 1 + 2k + (x_k < 0)): from
    // the cube, that of face hit; from axis a, the cube across its faces
    // (planes 0, 1), axis k across x_a = x_k with the sign of x_a (planes 2, 4)
    // and across x_a = -x_k with the other sign (planes 3, 5)
    const int kk = hit < 4 ? k1 : k2;
    const int across = in_cube ? 1 + hit : (hit < 2 ? 0 : 1 + 2 * kk + (neg ^ (hit & 1)));
    int reg_next = reg;
    if (tb < kInf) {
        const float n2 = next_candidate(C, tb);
        const int r2 = region_at(o, d, n2 < kInf ? 0.5f * (tb + n2) : 2.0f * tb + 1.0f);
        reg_next = r2 != reg ? r2 : across;
    }
    s.A = map_region(reg, make_float3(fmaf(ta, d.x, o.x), fmaf(ta, d.y, o.y), fmaf(ta, d.z, o.z)));
    const float3 B = segment_end(o, d, tb, reg);
    s.tb = tb;
    s.reg = reg;
    s.reg_next = reg_next;
    float3 e = make_float3(B.x - s.A.x, B.y - s.A.y, B.z - s.A.z);
    float len = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
    s.k = 0;
    // contracted segments are at most a few units long; anything else is a
    // degenerate ray (NaN / infinite end point) and contributes nothing
    if (!(len > 0.0f && len < 16.0f)) {
        s.n = 0;
        s.len = 0.0f;
        return;
    }
    float il = rcp(len);
    e.x *= il; e.y *= il; e.z *= il;
    s.e = e;
    s.len = len;
    s.n = (int)ceilf(len * istep);
    // rcp(+-0) = +-inf: the slab tests below then give +inf (or NaN, which
    // fminf ignores) for an axis the segment does not move along
    s.iex = rcp(e.x);
    s.iey = rcp(e.y);
    s.iez = rcp(e.z);
    s.doff = oct_stride * (uint32_t)((s.iex < 0.0f ? 1 : 0) | (s.iey < 0.0f ? 2 : 0) | (s.iez < 0.0f ? 4 : 0));
}

// Empty-space grid of the segment's octant at contracted point p.  Returns
// the byte D of p's cell: D > 0 means the cube of D cells a side with a
// corner at that cell, extending the way the segment travels, is empty; 0
// means the cell is occupied (the cube is the cell itself).  ue is the
// segment parameter at which the cube ends (slab test).
template <typename S>
__device__ __forceinline__ int dist_lookup(const S &sc, const Segment &s, float3 p, float &ue) {
    const int r = sc.dist_res;
    // cell of p: (p + 2) r / 4 rounded down (contracted points have p >= -2
    // up to rounding, so truncation is the floor), clamped to the grid
    const float os = sc.dist_scale, os2 = sc.dist_off;
    const int qx = cell_index(fmaf(p.x, os, os2), r);
    const int qy = cell_index(fmaf(p.y, os, os2), r);
    const int qz = cell_index(fmaf(p.z, os, os2), r);
    const int D = load_at<uint8_t>(sc.dist, s.doff + cell_offset(qx, qy, qz, r));
    const int ext = D > 0 ? D - 1 : 0;
    const float h = sc.dist_cell;
    const float bx = (float)(s.iex > 0.0f ? qx + ext + 1 : qx - ext) * h - 2.0f;
    const float by = (float)(s.iey > 0.0f ? qy + ext + 1 : qy - ext) * h - 2.0f;
    const float bz = (float)(s.iez > 0.0f ? qz + ext + 1 : qz - ext) * h - 2.0f;
    const float tx = (bx - s.A.x) * s.iex;
    const float ty = (by - s.A.y) * s.iey;
    const float tz = (bz - s.A.z) * s.iez;
    ue = fminf(tx, fminf(ty, tz));
    return D;
}

// Next lattice interval after leaving empty space at segment parameter
// uexit: the first whose midpoint lies past the exit, and at least k + 1.
__device__ __forceinline__ int skip_past(const Segment &s, float uexit, float istep) {
    const float kn = floorf((uexit - kSkipGuard) * istep - 0.5f) + 1.0f;
    // clamped to [0, n] (the float-to-int conversion saturates; NaN gives 0)
    const int knext = min((int)fmaxf(kn, 0.0f), s.n);
    return max(s.k + 1, knext);
}

// Pinhole ray through the centre of pixel (px, py) (unit direction).
__device__ __forceinline__ void pixel_ray(const DevCamera &cam, int px, int py, float3 &o, float3 &d) {
    const float vx = ((float)px + 0.5f - cam.cx) * cam.inv_fx;
    const float vy = ((float)py + 0.5f - cam.cy) * cam.inv_fy;
    d = make_float3(fmaf(cam.c2w[0], vx, fmaf(cam.c2w[1], vy, cam.c2w[2])),
                    fmaf(cam.c2w[4], vx, fmaf(cam.c2w[5], vy, cam.c2w[6])),
                    fmaf(cam.c2w[8], vx, fmaf(cam.c2w[9], vy, cam.c2w[10])));
    const float inv = __builtin_amdgcn_rsqf(d.x * d.x + d.y * d.y + d.z * d.z);
    d.x *= inv; d.y *= inv; d.z *= inv;
    o = make_float3(cam.c2w[3], cam.c2w[7], cam.c2w[11]);
}

// Camera of a launch tile: the last camera whose first tile is <= tile.
__device__ __forceinline__ int camera_of(const RenderBatch &rb, int tile) {
    int c = 0;
#pragma unroll
    for (int i = 1; i < kCamsPerLaunch; ++i)
        if (i < rb.n_cams && tile >= rb.cams[i].tile_start) c = i;
    return c;
}

// Deferred MLP (Eq. 3, App. B) for the 64 pixels of a wave on the matrix
// cores.  Each layer is computed transposed, H^T = W^T X^T, over 4 blocks of
// 16 pixels: the output of one layer (lane l holds hidden units 4(l/16) .. +3
// of pixel l % 16) is exactly the B operand the next layer needs, so only the
// input features and the final RGB pass through LDS.  A pixel is a column of
// every product, so inactive lanes cannot affect the others.
//   kPrec 0: fp32 inputs, v_mfma_f32_16x16x4f32 (K = 4 per instruction);
//   kPrec 1: fp16 inputs, v_mfma_f32_16x16x16f16 (K = 16);
//   kPrec 2: bf16 inputs, v_mfma_f32_16x16x16bf16_1k (K = 16).
// Accumulation, biases and ReLU are fp32 in every case.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
// LDS staging of the inputs, one row per pixel, sized so that four waves fit
// per SIMD (16 workgroups of one wave in a CU's 160 KB):
//   fp32: 36 floats (the 34 inputs zero-padded to nine K = 4 steps), row
//         stride 37 floats -- odd, so the 16 rows one instruction reads fall in
//         different banks;
//   fp16 / bf16: the inputs already converted, 48 halves (three K = 16
//         steps), row stride 52 halves = 26 banks, so the 16 eight-byte reads
//         of one instruction cover the 32 banks once.
// The outputs reuse the buffer as floats with the row stride kOut.
template <int kPrec>
struct MlpLds {
    static constexpr int kWidth = kPrec == 0 ? 36 : 48;      // inputs per row
    static constexpr int kStride = kPrec == 0 ? 37 : 52;     // elements per row
    static constexpr int kOut = kPrec == 0 ? 37 : 26;        // floats per row of the outputs
    static constexpr int kFloats = 64 * (kPrec == 0 ? 37 : 26);
};

__device__ __forceinline__ void mlp_encode(float *x, const Accum &acc, float3 d) {
    x[0] = acc.cd0; x[1] = acc.cd1; x[2] = acc.cd2;
    x[3] = acc.f0; x[4] = acc.f1; x[5] = acc.f2; x[6] = acc.f3;
    x[7] = d.x; x[8] = d.y; x[9] = d.z;
    // sin and cos of 2^k d, k = 0..3: the hardware sine and cosine at k = 0,
    // then the double-angle identities sin 2a = 2 sin a cos a and
    // cos 2a = 1 - 2 sin^2 a (three FP32 operations instead of two quarter-
    // rate transcendentals per term; the error stays near 1e-5 absolute)
    float sn[3] = {__sinf(d.x), __sinf(d.y), __sinf(d.z)};
    float cs[3] = {__cosf(d.x), __cosf(d.y), __cosf(d.z)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[10 + 3 * k + a] = sn[a];
            x[22 + 3 * k + a] = cs[a];
            const float s2 = 2.0f * sn[a];
            cs[a] = fmaf(-s2, sn[a], 1.0f);
            sn[a] = s2 * x[22 + 3 * k + a];
        }
    }
#pragma unroll
    for (int k = kMlpIn; k < 48; ++k) x[k] = 0.0f;
}

// Half-precision operand type of kPrec 1 (fp16) and 2 (bf16).
template <int kPrec>
using half4_t = typename std::conditional<kPrec == 1, halfx4, bf16x4>::type;
template <int kPrec>
using half_t = typename std::conditional<kPrec == 1, _Float16, __bf16>::type;

template <int kPrec>
__device__ __forceinline__ half4_t<kPrec> to_half4(const float v[4]) {
    using H = half_t<kPrec>;
    return half4_t<kPrec>{(H)v[0], (H)v[1], (H)v[2], (H)v[3]};
}

// 16x16 block product with K = 16 in half precision: lane l supplies
// A[l % 16][4(l/16) .. +3] and B[4(l/16) .. +3][l % 16].
template <int kPrec>
__device__ __forceinline__ floatx4 mfma16(half4_t<kPrec> a, half4_t<kPrec> b, floatx4 c) {
    if constexpr (kPrec == 1) return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Returns h(x) for this lane's pixel.  All 64 lanes must call it.
template <int kPrec>
__device__ __forceinline__ float3 deferred_mlp_mfma(const float *__restrict__ W, float *xs, const Accum &acc,
                                                    float3 d, int lane) {
    using Lds = MlpLds<kPrec>;
    const int j = lane & 15, g = lane >> 4;
    const float *W0 = W, *b0 = W0 + kMlpIn * kMlpHidden, *W1 = b0 + kMlpHidden, *b1 = W1 + kMlpHidden * kMlpHidden,
                *W2 = b1 + kMlpHidden, *b2 = W2 + kMlpHidden * kMlpOut;
    // Weights and biases first, so their loads overlap the input encoding.
    // Layer-1 A operand W0^T[hidden j][k]: fp32 steps take k = 9g + q,
    // half-precision steps k = 16 (q / 4) + 4g + q % 4; rows past the 34
    // inputs and output columns past 3 are zero (loaded from a valid address,
    // then replaced, so no load is conditional).
    constexpr int kA0 = kPrec == 0 ? 9 : 12;
    float a0[kA0], a1[4], a2[4], c0[4], c1[4];
#pragma unroll
    for (int q = 0; q < kA0; ++q) {
        const int k = kPrec == 0 ? 9 * g + q : 16 * (q >> 2) + 4 * g + (q & 3);
        const float v = W0[min(k, kMlpIn - 1) * kMlpHidden + j];
        a0[q] = k < kMlpIn ? v : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a1[q] = W1[(4 * g + q) * kMlpHidden + j];
        const float v = W2[(4 * g + q) * kMlpOut + min(j, kMlpOut - 1)];
        a2[q] = j < kMlpOut ? v : 0.0f;
        c0[q] = b0[4 * g + q];
        c1[q] = b1[4 * g + q];
    }
    {
        float x[48];
        mlp_encode(x, acc, d);
        if constexpr (kPrec == 0) {
#pragma unroll
            for (int i = 0; i < Lds::kWidth; ++i) xs[lane * Lds::kStride + i] = x[i];
        } else {
            half4_t<kPrec> *row = reinterpret_cast<half4_t<kPrec> *>(reinterpret_cast<half_t<kPrec> *>(xs) +
                                                                    lane * Lds::kStride);
#pragma unroll
            for (int i = 0; i < Lds::kWidth / 4; ++i) row[i] = to_half4<kPrec>(x + 4 * i);
        }
    }
    __syncthreads();
    // the four blocks of 16 pixels go through each layer together, so four
    // independent accumulation chains keep the matrix core busy
    floatx4 c[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) c[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (kPrec == 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                c[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[q], xs[(16 * mt + j) * Lds::kStride + 9 * g + q], c[mt],
                                                             0, 0, 0);
    } else {
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) {
            const half4_t<kPrec> a = to_half4<kPrec>(a0 + 4 * ks);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const half_t<kPrec> *xr = reinterpret_cast<const half_t<kPrec> *>(xs) + (16 * mt + j) * Lds::kStride;
                c[mt] = mfma16<kPrec>(a, *reinterpret_cast<const half4_t<kPrec> *>(xr + 16 * ks + 4 * g), c[mt]);
            }
        }
    }
    float h[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) h[mt][r] = fmaxf(c[mt][r] + c0[r], 0.0f);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) c[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (kPrec == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) c[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q], h[mt][q], c[mt], 0, 0, 0);
    } else {
        const half4_t<kPrec> a = to_half4<kPrec>(a1);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) c[mt] = mfma16<kPrec>(a, to_half4<kPrec>(h[mt]), c[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) h[mt][r] = fmaxf(c[mt][r] + c1[r], 0.0f);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) c[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (kPrec == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) c[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[q], h[mt][q], c[mt], 0, 0, 0);
    } else {
        const half4_t<kPrec> a = to_half4<kPrec>(a2);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) c[mt] = mfma16<kPrec>(a, to_half4<kPrec>(h[mt]), c[mt]);
    }
    __syncthreads();   // every lane has read its inputs; reuse xs for the outputs
    // output unit r of pixel 16 mt + j is c[mt][r] of lane j (g = 0)
    if (g == 0) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < kMlpOut; ++r) xs[(16 * mt + j) * Lds::kOut + r] = c[mt][r] + b2[r];
    }
    __syncthreads();
    return make_float3(xs[lane * Lds::kOut + 0], xs[lane * Lds::kOut + 1], xs[lane * Lds::kOut + 2]);
}

// Samples a lane may park ahead of its compositing, and the LDS of a wave:
// during the march the parking area (kQueue x 64 x (p, delta)), the results
// of one shading pass (64 x 8 floats, by shading slot) and the 64-entry
// shading map; the MLP staging afterwards.
constexpr int kQueue = 3;
constexpr int kParkFloats = 4 * 64 * kQueue + 8 * 64 + 64;
template <int kPrec>
constexpr int kLdsFloats = MlpLds<kPrec>::kFloats > kParkFloats ? MlpLds<kPrec>::kFloats : kParkFloats;

// kLevels: empty space is skipped with the occupancy levels themselves
// (skip_mode 1) instead of the distance grid (skip_mode 0).
// kMode: 0 renders; 1 also adds the statistics counters (and records the
// gathers when rb.rec is set); 2 also takes the phase profile.
// March parameters of one tile's rays.
struct TileParams {
    float step, istep, t_min;
    int32_t delta_mode;
};

// Measurement outputs of the statistics variants (kMode >= 1); see RenderBatch.
struct MeasureArgs {
    unsigned long long *stats;
    uint32_t *rec;
    int32_t *rec_count;
    int32_t rec_cap, total_tiles;
    unsigned long long *phases;
};

// One wave renders local tile lt of camera cam (launch tile `tile`, used by
// the measurement outputs only) of scene sc; lane = threadIdx.x.
template <int kMode, int kMlpPrec, int kFeat, bool kLevels, typename S, typename Cam>
__device__ __forceinline__ void render_tile(const S &sc, const Cam &cam, int lt, int tile,
                                            const TileParams tp, const MeasureArgs ma, float *lds, const int lane) {
    constexpr bool kStats = kMode >= 1, kPhase = kMode == 2;
    // the tile's corner is uniform: kept in scalar registers
    const int tx0 = __builtin_amdgcn_readfirstlane((lt % cam.tiles_x) * kTile);
    const int ty0 = __builtin_amdgcn_readfirstlane((lt / cam.tiles_x) * kTile);
    const int px = tx0 + (lane & (kTile - 1));
    const int py = ty0 + (lane / kTile);
    const bool active = px < cam.width && py < cam.height;
    PhaseClock<kPhase> ph;
    ph.start();

    // ---- pinhole ray
    float vx = ((float)px + 0.5f - cam.cx) * cam.inv_fx;
    float vy = ((float)py + 0.5f - cam.cy) * cam.inv_fy;
    float3 d = make_float3(fmaf(cam.c2w[0], vx, fmaf(cam.c2w[1], vy, cam.c2w[2])),
                           fmaf(cam.c2w[4], vx, fmaf(cam.c2w[5], vy, cam.c2w[6])),
                           fmaf(cam.c2w[8], vx, fmaf(cam.c2w[9], vy, cam.c2w[10])));
    float inv = __builtin_amdgcn_rsqf(d.x * d.x + d.y * d.y + d.z * d.z);
    d.x *= inv; d.y *= inv; d.z *= inv;
    const float3 o = make_float3(cam.c2w[3], cam.c2w[7], cam.c2w[11]);

    Counters cnt = {0u, 0u, 0u, 0u, 0u};
    Accum acc = {1.0f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float step = tp.step, istep = tp.istep;
    Segment s;
    {
        const Candidates C = make_candidates(o, d);
        const float c1 = next_candidate(C, 0.0f);
        open_segment(o, d, 0.0f, region_at(o, d, c1 < kInf ? 0.5f * c1 : 1.0f), istep, sc.dist_oct_stride, s);
    }
    int nseg = 1;
    bool alive = active, terminated = false;
    float known[kMaxLevels] = {0.0f, 0.0f, 0.0f, 0.0f};   // per level: occupied up to this u
    if (kPhase) ph.lap(kPhSetup);

    // The march runs ahead of the shading: every live lane finds up to kQueue
    // occupied samples (cheap skip iterations) and parks them in LDS; then the
    // wave shades up to 64 parked samples at once -- oldest first, whichever
    // lane's ray they belong to -- so the expensive gather-and-decode code
    // runs with as many lanes busy as possible; then every lane composites
    // its own shaded samples in ray order.  Samples parked past an early
    // termination are dropped, so the image is the one a one-sample-at-a-time
    // march gives.
    float4 *pq = reinterpret_cast<float4 *>(lds);             // [kQueue][64] parked (p, delta)
    float4 *rs = pq + kQueue * 64;                            // [64] x 2: results by shading slot
    // finite from the start: the branch-free compositing reads slot 0 for
    // lanes with nothing to composite
    rs[2 * lane] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
    rs[2 * lane + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int *imap = reinterpret_cast<int *>(rs + 2 * 64);          // [64] shading slot -> parked entry
    int pc = 0;                                               // samples parked by this lane
    while (__any(alive || pc > 0)) {
        if (kPhase) ph.count(kPhRounds);
        // ---- march: live lanes park up to kQueue samples, one step per
        // pass; the wave stops once 64 samples are parked (a round shades no
        // more), so slow lanes do not hold the others back.  Issue priority
        // by phase: a SIMD's waves that are shading go first, then those
        // compositing, then those marching or in the deferred MLP (the same
        // images; the frames are about 1% faster at 1080p and 2% at 4K)
        __builtin_amdgcn_s_setprio(0);
        for (;;) {
            const bool want = alive && pc < kQueue;
            int parked = 0;
#pragma unroll
            for (int j = 0; j < kQueue; ++j) parked += __popcll(__ballot(pc > j));
            if (!__any(want) || parked >= 64) break;
            if (kPhase) ph.count(kPhMarchPasses);
            // a lane whose segment is done spends this pass on the next
            // region's segment, if any
            const bool open = want && s.k >= s.n;
            if (kPhase ? __any(open) : true) {
                if (kPhase) ph.lap(kPhMarch);
                if (open) {
                    if (!(s.tb < kInf) || nseg >= 8) {
                        alive = false;
                    } else {
                        open_segment(o, d, s.tb, s.reg_next, istep, sc.dist_oct_stride, s);
                        ++nseg;
                        if (kStats) ++cnt.opens;
                        known[0] = known[1] = known[2] = known[3] = 0.0f;
                    }
                }
                if (kPhase) {
                    ph.lap(kPhOpen);
                    ph.count(kPhOpenPasses);
                }
            }
            if (!want || open) continue;
            // ---- one march step
            const float u0 = (float)s.k * step;
            const float u1 = fminf(u0 + step, s.len);
            const float um = 0.5f * (u0 + u1);
            const float3 p = make_float3(fmaf(um, s.e.x, s.A.x), fmaf(um, s.e.y, s.A.y), fmaf(um, s.e.z, s.A.z));
            if (kStats) ++cnt.visited;
            // empty >= 0: the sample is in empty space, which the segment
            // leaves at parameter uexit.  A cell seen occupied stays known
            // until the segment leaves it (its exit minus the guard), so later
            // samples inside it need no lookup.
            int empty = -1;
            float uexit = 0.0f;
            if constexpr (!kLevels) {
                // empty-space grid: leave the whole empty cube ahead, or
                // remember the occupied cell
                if (!(um < known[0])) {
                    if (kStats) ++cnt.occ_lookups;
                    float ue;
                    const int D = dist_lookup(sc, s, p, ue);
                    if (D == 0) {
                        known[0] = ue - kSkipGuard;
                    } else {
                        empty = 0;
                        uexit = ue;
                    }
                }
            } else {
                // the occupancy levels, coarse to fine: stop at the first
                // empty level and leave its cell
#pragma unroll
                for (int l = 0; l < kMaxLevels; ++l) {
                    if (l < sc.occ_levels && empty < 0 && !(um < known[l])) {
                        const int rl = sc.occ_res[l];
                        const float os = (float)rl * 0.25f, os2 = 2.0f * os;
                        const int qx = cell_index(fmaf(p.x, os, os2), rl);
                        const int qy = cell_index(fmaf(p.y, os, os2), rl);
                        const int qz = cell_index(fmaf(p.z, os, os2), rl);
                        if (kStats) ++cnt.occ_lookups;
                        const bool occ = load_at<uint8_t>(sc.occ[l], cell_offset(qx, qy, qz, rl)) != 0;
                        // exit parameter of this cell along the segment (slab test)
                        const float h = sc.occ_cell[l];
                        const float bx = (float)(s.iex > 0.0f ? qx + 1 : qx) * h - 2.0f;
                        const float by = (float)(s.iey > 0.0f ? qy + 1 : qy) * h - 2.0f;
                        const float bz = (float)(s.iez > 0.0f ? qz + 1 : qz) * h - 2.0f;
                        const float tx = (bx - s.A.x) * s.iex;
                        const float ty = (by - s.A.y) * s.iey;
                        const float tz = (bz - s.A.z) * s.iez;
                        const float ue = fminf(tx, fminf(ty, tz));
                        if (occ) {
                            known[l] = ue - kSkipGuard;
                        } else {
                            empty = l;
                            uexit = ue;
                        }
                    }
                }
            }
            if (empty < 0) {
                float delta = u1 - u0;
                if (tp.delta_mode == 1) {
                    float3 y0 = make_float3(fmaf(u0, s.e.x, s.A.x), fmaf(u0, s.e.y, s.A.y), fmaf(u0, s.e.z, s.A.z));
                    float3 y1 = (s.k == s.n - 1)
                                    ? segment_end(o, d, s.tb, s.reg)
                                    : make_float3(fmaf(u1, s.e.x, s.A.x), fmaf(u1, s.e.y, s.A.y), fmaf(u1, s.e.z, s.A.z));
                    bool at_inf = false;
                    if (s.reg != 0) {
                        const int jj = (s.reg - 1) >> 1;
                        const float sg = ((s.reg - 1) & 1) ? -1.0f : 1.0f;
                        const float y1j = jj == 0 ? y1.x : (jj == 1 ? y1.y : y1.z);
                        at_inf = sg * y1j >= 2.0f;
                    }
                    if (at_inf) {
                        delta = kInf;
                    } else {
                        float3 x0 = unmap_region(s.reg, y0), x1 = unmap_region(s.reg, y1);
                        float dx = x1.x - x0.x, dy = x1.y - x0.y, dz = x1.z - x0.z;
                        delta = sqrtf(dx * dx + dy * dy + dz * dz);
                    }
                }
                pq[pc * 64 + lane] = make_float4(p.x, p.y, p.z, delta);
                ++pc;
                ++s.k;
            } else {
                // leave the empty cell: first lattice interval whose midpoint
                // lies past the exit
                s.k = skip_past(s, uexit, istep);
            }
        }
        if (kPhase) ph.lap(kPhMarch);
        // ---- shade: parked samples numbered level by level (all first
        // samples, then all second ones ...), lane order within a level;
        // slots past 64 wait for the next round
        int total = 0;
#pragma unroll
        for (int j = 0; j < kQueue; ++j) {
            const int item = total + lanes_below(__ballot(pc > j));
            if (pc > j && item < 64) imap[item] = j * 64 + lane;
            total += __popcll(__ballot(pc > j));
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(2);
        if (lane < total) {
            const int e = imap[lane];
            const float4 q = pq[e];
            const SampleResult r = eval_sample<kFeat>(sc, make_float3(q.x, q.y, q.z), q.w);
            rs[2 * lane] = make_float4(r.trans, r.sg[0], r.sg[1], r.sg[2]);
            rs[2 * lane + 1] = make_float4(r.sg[3], r.sg[4], r.sg[5], r.sg[6]);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(1);
        if (kPhase) {
            ph.lap(kPhShade);
            ph.count(kPhShadePasses, total > 0 ? 1 : 0);
            ph.count(kPhShadeLanes, (uint32_t)min(total, 64));
        }
        // ---- composite this lane's shaded samples in ray order
        int done = 0, before = 0;
#pragma unroll
        for (int j = 0; j < kQueue; ++j) {
            const int item = before + lanes_below(__ballot(pc > j));
            before += __popcll(__ballot(pc > j));
            if constexpr (!kStats) {
                // branch-free: an unused slot reads the result area at item 0
                // (always finite) and contributes with weight 0, which leaves
                // every accumulator bit for bit unchanged (the branch around
                // the update made the compiler copy the accumulators)
                const bool use = j < pc && item < 64 && !terminated;
                const int it = use ? item : 0;
                const float4 ra = rs[2 * it], rbv = rs[2 * it + 1];
                const float alpha = use ? 1.0f - ra.x : 0.0f;
                const float wt = acc.T * alpha;
                acc.cd0 = fmaf(wt, ra.y, acc.cd0);
                acc.cd1 = fmaf(wt, ra.z, acc.cd1);
                acc.cd2 = fmaf(wt, ra.w, acc.cd2);
                acc.f0 = fmaf(wt, rbv.x, acc.f0);
                acc.f1 = fmaf(wt, rbv.y, acc.f1);
                acc.f2 = fmaf(wt, rbv.z, acc.f2);
                acc.f3 = fmaf(wt, rbv.w, acc.f3);
                acc.T *= use ? ra.x : 1.0f;
                done += use ? 1 : 0;
                if (use && acc.T < tp.t_min) {   // early termination (Sec. 6)
                    alive = false;
                    terminated = true;
                }
            } else if (j < pc && item < 64 && !terminated) {
                const int e = j * 64 + lane;
                if (kStats && ma.rec) {
                    // measurement: record the texel offsets of this sample
                    const uint32_t k = cnt.evaluated;
                    if (k < (uint32_t)ma.rec_cap) {
                        const float4 q = pq[e];
                        const Footprint f = footprint(sc, make_float3(q.x, q.y, q.z));
                        const uint32_t qs = (uint32_t)tile * 64u + (uint32_t)lane;
                        *reinterpret_cast<u32x4 *>(ma.rec + 4 * ((size_t)k * (size_t)ma.total_tiles * 64u + qs)) =
                            u32x4{f.op[0], f.op[1], f.op[2], (f.bi << 13) | f.ol};
                    }
                }
                const float4 ra = rs[2 * item], rbv = rs[2 * item + 1];
                const SampleResult r = {ra.x, {ra.y, ra.z, ra.w, rbv.x, rbv.y, rbv.z, rbv.w}};
                composite<kStats>(acc, r, cnt);
                ++done;
                if (acc.T < tp.t_min) {          // early termination (Sec. 6)
                    alive = false;
                    terminated = true;
                }
            }
        }
        // ---- keep the samples not shaded yet, in order
        if (terminated) {
            pc = 0;
        } else if (done > 0) {
#pragma unroll
            for (int j = 0; j + 1 < kQueue; ++j)
                if (j + done < pc) pq[j * 64 + lane] = pq[(j + done) * 64 + lane];
            pc -= done;
        }
        __syncthreads();
        if (kPhase) ph.lap(kPhComposite);
    }

    __builtin_amdgcn_s_setprio(0);      // the MLP at the marching waves' priority
    const float3 h = deferred_mlp_mfma<kMlpPrec>(sc.mlp, lds, acc, d, lane);
    if (active) {
        // the pixel again from the lane id (an opaque copy, so the compiler
        // recomputes it instead of holding px and py through the march)
        int l2 = lane;
        asm volatile("" : "+v"(l2));
        const int ox = tx0 + (l2 & (kTile - 1));
        const int oy = ty0 + (l2 / kTile);
        float4 rgba = make_float4(acc.cd0 + h.x, acc.cd1 + h.y, acc.cd2 + h.z, 1.0f - acc.T);
        *reinterpret_cast<float4 *>(cam.out + ((int64_t)oy * cam.width + ox) * 4) = rgba;
    }
    if (kPhase) ph.lap(kPhMlp);
    if (kStats && ma.rec_count) ma.rec_count[tile * 64 + lane] = (int32_t)cnt.evaluated;
    if (kStats) {
        unsigned long long v[6] = {active ? 1ull : 0ull, cnt.occ_lookups, cnt.visited, cnt.evaluated, cnt.contributing,
                                   terminated ? 1ull : 0ull};
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            unsigned long long x = v[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            if (lane == 0 && x) atomicAdd(ma.stats + i, x);
        }
        if (kPhase) {
            ph.count(kPhWaves);
            uint32_t x = cnt.opens;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            ph.count(kPhOpenLanes, x);
            if (lane < kPhSlots && ph.v) atomicAdd(ma.phases + lane, (unsigned long long)ph.v);
        }
    }
}

template <int kMode, int kMlpPrec, int kFeat, bool kLevels>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_render(const DevScene sc, const RenderBatch rb) {
    __shared__ float lds[kLdsFloats<kMlpPrec>];
    const int slot = xcd_remap((int)blockIdx.x, rb.total_tiles);
    int tile = rb.order ? rb.order[slot] : slot;
    if ((unsigned)tile >= (unsigned)rb.total_tiles) tile = slot;   // never leave the launch
    int c = 0;
#pragma unroll
    for (int i = 1; i < kCamsPerLaunch; ++i)
        if (i < rb.n_cams && tile >= rb.cams[i].tile_start) c = i;
    const DevCamera &cam = rb.cams[c];
    const TileParams tp = {rb.step, rb.inv_step, rb.t_min, rb.delta_mode};
    const MeasureArgs ma = {rb.stats, rb.rec, rb.rec_count, rb.rec_cap, rb.total_tiles, rb.phases};
    render_tile<kMode, kMlpPrec, kFeat, kLevels>(sc, cam, tile - cam.tile_start, tile, tp, ma, lds,
                                                    (int)threadIdx.x);
}

// Served launch: workgroup b renders position b / 8 of its XCD's share of
// the launch (XCD x = blockIdx % 8 holds the runs of kXcdChunk consecutive
// tiles that xcd_remap deals to x), so neighbouring tiles still share an L2.
// The grid is a fixed class (the server captures one graph per class), the
// smallest that gives every tile a workgroup of its own; workgroups past the
// launch's tiles exit at once.  A launch larger than the largest such class
// is persistent (a grid of the device's wave slots): its workgroups go on
// taking positions from the XCD's counter, asking for the next one as they
// start each tile so that the atomic's round trip overlaps the render, until
// the share is exhausted; the counters are zeroed before such a launch
// (k_zero_ctl).  (A 4096-workgroup persistent grid rendered a 1080p request
// 13% slower than one workgroup per tile, and 5% slower once its workgroups
// no longer counted themselves out on one shared counter at the end.)  Each
// tile belongs to one request, which names its camera, march parameters and
// scene (a slot of the server's scene table).
typedef const __attribute__((address_space(4))) DevScene ConstScene;
typedef const __attribute__((address_space(4))) ServeLaunch ConstLaunch;
typedef const __attribute__((address_space(4))) ServeWork ConstWork;

__device__ __forceinline__ int xcd_share_tile(int x, uint32_t i) {
    return (int)((((i / kXcdChunk) * kXcds + (uint32_t)x) * kXcdChunk) + i % kXcdChunk);
}

// The scene table and the launch descriptors are read through the constant
// address space: they do not change during the launch, so the compiler reads
// them with scalar loads and may repeat a load instead of holding its value.
template <int kMlpPrec, int kFeat, bool kLevels>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_render_served(
    ConstScene *__restrict__ table, ConstLaunch *__restrict__ launch, ServeCtl *__restrict__ ctl) {
    __shared__ float lds[kLdsFloats<kMlpPrec>];
    const int x = (int)(blockIdx.x % kXcds);
    const uint32_t base = gridDim.x / kXcds;      // positions handed out by workgroup index
    uint32_t *counter = ctl->next + x * kCtlStride;
    uint32_t i = blockIdx.x / kXcds;
    // a launch with more positions per XCD than the grid gives it loops
    const bool loops = base < (uint32_t)((launch->total_tiles + kXcds - 1) / kXcds);
    for (;;) {
        // nothing is carried from one tile to the next: opaque copies of the
        // lane id and the launch pointer keep the compiler from hoisting
        // lane-only address arithmetic and descriptor loads out of this loop
        // and holding them in registers through every tile
        // (the lane id is recomputed from the exec mask: a workgroup is one wave)
        int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        ConstLaunch *L = launch;
        asm volatile("" : "+v"(lane), "+s"(L));
        const int n = L->total_tiles, nw = L->n_work;
        const int tile = xcd_share_tile(x, i);
        if (i >= (uint32_t)n || tile >= n) break;
        uint32_t nx = 0;                           // the next position, in flight during the render
        if (loops && lane == 0) nx = base + atomicAdd(counter, 1u);
        int c = 0;
#pragma unroll
        for (int k = 1; k < kCamsPerLaunch; ++k)
            if (k < nw && tile >= L->work[k].cam.tile_start) c = k;
        ConstWork &w = L->work[c];
        const TileParams tp = {w.step, w.inv_step, w.t_min, w.delta_mode};
        const MeasureArgs ma = {nullptr, nullptr, nullptr, 0, 0, nullptr};
        render_tile<0, kMlpPrec, kFeat, kLevels>(table[w.scene], w.cam, tile - w.cam.tile_start, tile, tp, ma, lds,
                                                    lane);
        if (!loops) break;
        __syncthreads();
        i = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(nx, 0, 64));
    }
}

// Zero a served launch's counters (a node of its own before the launch, so
// that no workgroup of the launch has to find out that it is the last one).
__global__ __launch_bounds__(64) void k_zero_ctl(ServeCtl *__restrict__ ctl) {
    if ((int)threadIdx.x < kXcds) ctl->next[threadIdx.x * kCtlStride] = 0u;
}

// Tile cost for the launch order.  kCostRays rays of every 8x8 tile (pixels
// (2,2), (5,2), (2,5) and (5,5) of the tile, clamped to the image) march as
// the renderer does, through empty space to their first occupied sample.
// With kEffort they go on through occupied space, where the opacity of each
// evaluated sample (its density; the rest of the shading is not needed) is
// composited, until the ray terminates (T < t_min), ends, or has evaluated
// kCostEval samples.  The effort E of a tile is the sum of its rays'
// evaluated samples (a march still running after kCostSteps steps counts
// one); its key is 0 for E = 0 and 1 + [E >= 2 kCostRays] +
// [E >= 3 kCostRays] + [E >= 4 kCostRays] otherwise: rays that reach no
// occupied space only march, rays that terminate within a sample or two
// shade little, and rays that keep shading cost the most.  Without kEffort
// the key is the number of rays that reach occupied space (the cheaper
// prepass, for launches so large that the end of the launch is a small part
// of it).
constexpr int kCostSteps = 64;
constexpr int kCostEval = 4;
constexpr int kEffortMaxTiles = 1 << 16;
constexpr int kGroupTiles = 64 / kCostRays;                   // tiles of one k_tile_cost wave
constexpr int kCountBits = kGroupTiles < 32 ? 5 : 7;           // a group's count of one key
constexpr int kScanBits = 64 / kCostKeys;                      // a workgroup's count of one key
static_assert(kCostKeys * kCountBits <= 32 && (uint64_t)64 * kGroupTiles < (1ull << kScanBits), "count fields");
template <bool kEffort>
__global__ __launch_bounds__(64) void k_tile_cost(const DevScene sc, const RenderBatch rb, uint8_t *__restrict__ keys,
                                                  uint32_t *__restrict__ group_counts) {
    const int g = (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int tile = g / kCostRays, sub = g % kCostRays;
    int ev = 0;                                               // samples this ray evaluated
    if (tile < rb.total_tiles) {
        const DevCamera &cam = rb.cams[camera_of(rb, tile)];
        const int lt = tile - cam.tile_start;
        const int px = min((lt % cam.tiles_x) * kTile + (kCostRays == 1 ? 4 : (sub & 1) ? 5 : 2), cam.width - 1);
        const int py = min((lt / cam.tiles_x) * kTile + (kCostRays == 1 ? 4 : (sub & 2) ? 5 : 2), cam.height - 1);
        float3 o, d;
        pixel_ray(cam, px, py, o, d);
        const float step = rb.step, istep = rb.inv_step;
        Segment s;
        const Candidates C = make_candidates(o, d);
        const float c1 = next_candidate(C, 0.0f);
        open_segment(o, d, 0.0f, region_at(o, d, c1 < kInf ? 0.5f * c1 : 1.0f), istep, sc.dist_oct_stride, s);
        int nseg = 1, it = 0;
        float T = 1.0f;
        for (; it < kCostSteps; ++it) {
            if (s.k >= s.n) {
                if (!(s.tb < kInf) || nseg >= 8) break;
                open_segment(o, d, s.tb, s.reg_next, istep, sc.dist_oct_stride, s);
                ++nseg;
                continue;
            }
            const float u0 = (float)s.k * step;
            const float u1 = fminf(u0 + step, s.len);
            const float um = 0.5f * (u0 + u1);
            const float3 p = make_float3(fmaf(um, s.e.x, s.A.x), fmaf(um, s.e.y, s.A.y), fmaf(um, s.e.z, s.A.z));
            float ue;
            if (dist_lookup(sc, s, p, ue) == 0) {
                // an occupied sample: the renderer evaluates it
                if (!kEffort) {
                    ev = 1;
                    break;
                }
                T *= eval_sample<0>(sc, p, u1 - u0).trans;
                if (++ev >= kCostEval || T < rb.t_min) break;
                ++s.k;
            } else {
                s.k = skip_past(s, ue, istep);
            }
        }
        if (it == kCostSteps && ev == 0) ev = 1;
    }
    // the kCostRays rays of a tile are consecutive lanes: their effort from
    // the bits of ev (at most kCostEval < 8)
    static_assert(kCostEval < 8 && kCostRays * kCostEval < 256, "effort bits");
    const uint64_t tm = ((1ull << kCostRays) - 1) << ((int)threadIdx.x & ~(kCostRays - 1));
    int key;
    if (kEffort) {
        int effort = 0;
#pragma unroll
        for (int bit = 0; bit < 3; ++bit) effort += __popcll(__ballot((ev >> bit) & 1) & tm) << bit;
        key = effort == 0 ? 0 : 1 + (effort >= 2 * kCostRays) + (effort >= 3 * kCostRays) + (effort >= 4 * kCostRays);
    } else {
        key = __popcll(__ballot(ev > 0) & tm);
    }
    const bool head = tile < rb.total_tiles && sub == 0;
    if (head) keys[tile] = (uint8_t)key;
    // the keys of the wave's kGroupTiles tiles (a group), counted per key in
    // kCountBits-bit fields
    uint32_t packed = 0u;
#pragma unroll
    for (int k = 0; k < kCostKeys; ++k) packed |= (uint32_t)__popcll(__ballot(head && key == k)) << (kCountBits * k);
    if (threadIdx.x == 0) group_counts[blockIdx.x] = packed;
}

// Stable counting sort of a launch's tiles by cost key, highest key first.
// A wave of k_tile_cost covers a group of kGroupTiles consecutive tiles and
// counts their keys.  Here a 64-lane workgroup places 64 groups, a lane per
// group: the lanes sum the counts of all groups (the totals) and of the
// groups before the workgroup's first, a scan over the lanes adds the counts
// of the lower lanes' groups, and each lane then writes its tiles' positions
// in ascending tile order.  Small workgroups find free wave slots while a
// render kernel occupies the device.
constexpr int kOrderLoads = 16;                               // group counts in flight per lane
__global__ __launch_bounds__(64) void k_tile_order(const uint8_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ group_counts, int n,
                                                   int32_t *__restrict__ order) {
    const int lane = (int)threadIdx.x;
    const int ngroups = (n + kGroupTiles - 1) / kGroupTiles;
    const int g0 = (int)blockIdx.x * 64;                      // first group of this workgroup
    int total[kCostKeys], before[kCostKeys];
#pragma unroll
    for (int k = 0; k < kCostKeys; ++k) total[k] = before[k] = 0;
    for (int base = 0; base < ngroups; base += 64 * kOrderLoads) {
        uint32_t w[kOrderLoads];
#pragma unroll
        for (int u = 0; u < kOrderLoads; ++u) {
            const int g = base + 64 * u + lane;
            w[u] = g < ngroups ? group_counts[g] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kOrderLoads; ++u) {
            const bool earlier = base + 64 * u + lane < g0;
#pragma unroll
            for (int k = 0; k < kCostKeys; ++k) {
                const int c = (int)((w[u] >> (kCountBits * k)) & ((1u << kCountBits) - 1u));
                total[k] += c;
                before[k] += earlier ? c : 0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kCostKeys; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            total[k] += __shfl_xor(total[k], off, 64);
            before[k] += __shfl_xor(before[k], off, 64);
        }
    }
    // this lane's group: its counts widened to kScanBits-bit fields and
    // scanned over the lanes
    const int g = g0 + lane;
    const uint32_t mine = g < ngroups ? group_counts[g] : 0u;
    uint64_t x = 0;
#pragma unroll
    for (int k = 0; k < kCostKeys; ++k)
        x |= (uint64_t)((mine >> (kCountBits * k)) & ((1u << kCountBits) - 1u)) << (kScanBits * k);
    uint64_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const uint64_t excl = incl - x;
    // first position of each key for this lane's tiles: all tiles of heavier
    // keys, then those of the same key in earlier groups
    int pos[kCostKeys];
    int run = 0;
#pragma unroll
    for (int k = kCostKeys - 1; k >= 0; --k) {
        pos[k] = run + before[k] + (int)((excl >> (kScanBits * k)) & ((1ull << kScanBits) - 1ull));
        run += total[k];
    }
    if (g < ngroups) {
        u32x4 kv[kGroupTiles / 16];
#pragma unroll
        for (int v = 0; v < kGroupTiles / 16; ++v)
            kv[v] = *reinterpret_cast<const u32x4 *>(keys + kGroupTiles * g + 16 * v);
#pragma unroll
        for (int j = 0; j < kGroupTiles; ++j) {
            const int i = kGroupTiles * g + j;
            const int key = (int)byte_of(kv[j >> 4][(j >> 2) & 3], j & 3);
            int at = pos[0];
#pragma unroll
            for (int k = 1; k < kCostKeys; ++k) at = key == k ? pos[k] : at;
            if (i < n) order[at] = i;
#pragma unroll
            for (int k = 0; k < kCostKeys; ++k) pos[k] += key == k ? 1 : 0;
        }
    }
}

__global__ void k_identity_order(int32_t *__restrict__ order, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) order[i] = i;
}

// Gather replay (measurement only): each lane re-issues, round by round, the
// texel loads the renderer made for its pixel -- the brick slot, then the six
// plane pairs and the four brick pairs -- with the same tile order and wave
// shape, and no arithmetic beyond the addresses.  Its time bounds what the
// renderer's gathers alone can reach on this working set.
__global__ __launch_bounds__(64) void k_gather_replay(const DevScene sc, const uint32_t *__restrict__ rec,
                                                      const int32_t *__restrict__ rec_count, int cap,
                                                      const int32_t *__restrict__ order, int total_tiles,
                                                      float *__restrict__ out) {
    const int slot = xcd_remap((int)blockIdx.x, total_tiles);
    int tile = order ? order[slot] : slot;
    if ((unsigned)tile >= (unsigned)total_tiles) tile = slot;   // an order of another launch
    const uint32_t q = (uint32_t)tile * 64u + threadIdx.x;
    const size_t slots = (size_t)total_tiles * 64u;
    const int n = min(rec_count[q], cap);
    const uint32_t prow = (uint32_t)sc.R * kChannels;
    uint32_t sink = 0u;
    for (int k = 0; __any(k < n); ++k) {
        if (k < n) {
            const u32x4 r = *reinterpret_cast<const u32x4 *>(rec + 4 * ((size_t)k * slots + q));
            const int brick = load_at<int>(reinterpret_cast<const uint8_t *>(sc.brick_index), (r.w >> 13) * 4u);
            Texels x;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const uint32_t o = pl == 0 ? r.x : (pl == 1 ? r.y : r.z);
                x.t[2 * pl] = load_pair(sc.planes, o);
                x.t[2 * pl + 1] = load_pair(sc.planes, o + prow);
            }
            constexpr uint32_t sy = kBrick * kChannels, sz = kBrick * kBrick * kChannels;
            const uint32_t ob = (uint32_t)brick * kBrickBytes + (r.w & 8191u);
            x.g[0] = load_pair(sc.bricks, ob);
            x.g[1] = load_pair(sc.bricks, ob + sy);
            x.g[2] = load_pair(sc.bricks, ob + sz);
            x.g[3] = load_pair(sc.bricks, ob + sz + sy);
            asm volatile("" : "+v"(x.t[0]), "+v"(x.t[1]), "+v"(x.t[2]), "+v"(x.t[3]), "+v"(x.t[4]), "+v"(x.t[5]),
                         "+v"(x.g[0]), "+v"(x.g[1]), "+v"(x.g[2]), "+v"(x.g[3]));
            sink ^= x.t[0].x ^ x.g[0].x;
        }
    }
    reinterpret_cast<float4 *>(out)[q] = make_float4((float)n, (float)(sink & 1u), 0.0f, 0.0f);
}

// Eq. 8 dequantisation of a buffer of codes.  prec 1 runs deq_f16, the
// routine the fp16-feature render path applies to every code it reads, with
// the scale a the upload computes for that path.  prec 0 gives the correctly
// rounded float32 value (deq_f32) and prec 2 that value rounded again to
// bfloat16, which is the correctly rounded bfloat16 value, because k/255
// never lies within half a float32 ulp of a bfloat16 rounding boundary (its
// binary expansion repeats with period 8); the test-suite checks all codes.
__global__ void k_dequant(const uint8_t *__restrict__ codes, int64_t n, float m, float a, int prec,
                          void *__restrict__ out) {
    const float m2 = 2.0f * m, m255 = 255.0f * m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (prec == 1) {
            const _Float16 code = as_f16x2((uint32_t)codes[i]).x;     // the subnormal b 2^-24
            reinterpret_cast<__half *>(out)[i] = __float2half_rn(deq_f16(code, a * 16777216.0f, m));
        } else {
            const float v = deq_f32(codes[i], m2, m255);
            if (prec == 0) reinterpret_cast<float *>(out)[i] = v;
            else reinterpret_cast<__hip_bfloat16 *>(out)[i] = __float2bfloat16(v);
        }
    }
}

}  // namespace

template <int kMode, int kFeat, bool kLevels>
const void *render_kernel_mlp(int mlp_prec) {
    return mlp_prec == 0 ? (const void *)k_render<kMode, 0, kFeat, kLevels>
         : mlp_prec == 1 ? (const void *)k_render<kMode, 1, kFeat, kLevels>
                         : (const void *)k_render<kMode, 2, kFeat, kLevels>;
}

template <int kMode, bool kLevels>
const void *render_kernel_feat(const RenderBatch &rb) {
    return rb.feat_prec == 2 ? render_kernel_mlp<kMode, 2, kLevels>(rb.mlp_prec)
         : rb.feat_prec == 1 ? render_kernel_mlp<kMode, 1, kLevels>(rb.mlp_prec)
                             : render_kernel_mlp<kMode, 0, kLevels>(rb.mlp_prec);
}

template <int kMode>
const void *render_kernel_mode(const RenderBatch &rb) {
    return rb.skip_mode ? render_kernel_feat<kMode, true>(rb) : render_kernel_feat<kMode, false>(rb);
}

const void *render_kernel(const RenderBatch &rb) {
    if (rb.phases) return render_kernel_mode<2>(rb);
    if (rb.stats) return render_kernel_mode<1>(rb);
    return render_kernel_mode<0>(rb);
}

dim3 render_grid(const RenderBatch &rb) { return dim3((unsigned)rb.total_tiles); }

template <int kFeat, bool kLevels>
const void *served_kernel_mlp(int mlp_prec) {
    return mlp_prec == 0 ? (const void *)k_render_served<0, kFeat, kLevels>
         : mlp_prec == 1 ? (const void *)k_render_served<1, kFeat, kLevels>
                         : (const void *)k_render_served<2, kFeat, kLevels>;
}

const void *served_kernel(int mlp_prec, int feat_prec, int skip_mode) {
    if (feat_prec == 2) return skip_mode ? served_kernel_mlp<2, true>(mlp_prec) : served_kernel_mlp<2, false>(mlp_prec);
    if (feat_prec == 1) return skip_mode ? served_kernel_mlp<1, true>(mlp_prec) : served_kernel_mlp<1, false>(mlp_prec);
    return skip_mode ? served_kernel_mlp<0, true>(mlp_prec) : served_kernel_mlp<0, false>(mlp_prec);
}

hipError_t launch_zero_ctl(ServeCtl *ctl, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(64), 0, stream, ctl);
    return hipGetLastError();
}

hipError_t launch_render_served(const DevScene *table, const ServeLaunch *launch, ServeCtl *ctl, int mlp_prec,
                                int feat_prec, int skip_mode, int grid, hipStream_t stream) {
    if (grid < kXcds || grid % kXcds != 0) return hipErrorInvalidValue;
    ConstScene *t = (ConstScene *)table;
    ConstLaunch *l = (ConstLaunch *)launch;
    void *args[] = {&t, &l, &ctl};
    return hipLaunchKernel(served_kernel(mlp_prec, feat_prec, skip_mode), dim3((unsigned)grid), dim3(kRenderBlock),
                           args, 0, stream);
}

hipError_t launch_render(const DevScene &sc, const RenderBatch &rb, hipStream_t stream) {
    if (rb.total_tiles <= 0) return hipSuccess;
    void *args[] = {const_cast<DevScene *>(&sc), const_cast<RenderBatch *>(&rb)};
    return hipLaunchKernel(render_kernel(rb), render_grid(rb), dim3(kRenderBlock), args, 0, stream);
}

hipError_t launch_tile_order(const DevScene &sc, const RenderBatch &rb, uint8_t *keys, uint32_t *group_counts,
                             int32_t *order, hipStream_t stream) {
    if (rb.total_tiles <= 0 || rb.total_tiles > kOrderMaxTiles) return hipErrorInvalidValue;
    const int groups = (rb.total_tiles + kGroupTiles - 1) / kGroupTiles;
    if (rb.total_tiles <= kEffortMaxTiles)
        hipLaunchKernelGGL(k_tile_cost<true>, dim3((unsigned)groups), dim3(64), 0, stream, sc, rb, keys, group_counts);
    else
        hipLaunchKernelGGL(k_tile_cost<false>, dim3((unsigned)groups), dim3(64), 0, stream, sc, rb, keys, group_counts);
    hipLaunchKernelGGL(k_tile_order, dim3((unsigned)((groups + 63) / 64)), dim3(64), 0, stream, keys, group_counts,
                       rb.total_tiles, order);
    return hipGetLastError();
}

hipError_t launch_identity_order(int32_t *order, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_identity_order, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, order, n);
    return hipGetLastError();
}

hipError_t launch_gather_replay(const DevScene &sc, const uint32_t *rec, const int32_t *rec_count, int cap,
                                const int32_t *order, int total_tiles, float *out, hipStream_t stream) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_replay, dim3((unsigned)total_tiles), dim3(64), 0, stream, sc, rec, rec_count, cap,
                       order, total_tiles, out);
    return hipGetLastError();
}

hipError_t launch_dequant(const uint8_t *codes, int64_t n, float m, float a, int prec, void *out,
                          hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_dequant, dim3((unsigned)blocks), dim3(256), 0, stream, codes, n, m, a, prec, out);
    return hipGetLastError();
}

}  // namespace merf
