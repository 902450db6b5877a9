// wcl_common.h -- shared definitions of the MI355X Wilson-Clover library:
// lattice geometry of the blocked even/odd layout, storage formats, complex
// arithmetic and the gamma-projection tables of the chiral basis.
//
// Layout of every internal field ("blocked even/odd"): the lattice is tiled by
// hypercubes of extent tile[mu] (even, dividing L[mu]); these tiles are also
// the cores of the Schwarz blocks.  A site of parity p (= (x+y+z+t) mod 2) has
// half index h = tile_id * Hb + l/2, where tile_id is the lexicographic index
// of its tile, l the lexicographic index inside the tile and Hb the number of
// sites of one parity per tile.  Consecutive threads therefore read
// consecutive sites of one tile, and a Schwarz core is one contiguous range.
//
// Storage (structure of arrays, the site index innermost, one parity):
//   spinor   double : double2 [12][Vh]      complex component i = spin*3+colour
//            float  : float4  [6][Vh]       components (2k, 2k+1)
//            half   : uint4   [3][Vh]       components (4k .. 4k+3) as 8 halves
//   links    double : double2 [4 mu][2 p][9][Vh]   row-major 3x3
//            float  : float4  [4][2][4][Vh] (reals 0..15) + float2 [4][2][Vh]
//            half   : uint4   [4][2][2][Vh] (reals 0..15) + uint32 [4][2][Vh]
//   clover   double : double2 [2 p][36][Vh]
//            float  : float4  [2 p][18][Vh]
//            half   : uint4   [2 p][9][Vh]
//   A clover site holds two Hermitian 6x6 chirality blocks (spins 0,1 and
//   2,3), each packed as 6 real diagonal entries followed by the 15 complex
//   entries above the diagonal in row-major order: 36 reals per block.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#define WCL_HD __host__ __device__ __forceinline__
#define WCL_D __device__ __forceinline__

namespace wcl {

// ---------------------------------------------------------------------------
// Division by an invariant integer (Granlund & Montgomery 1994): for
// n < 2^31, q = (umulhi(n, m) + n) >> s with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) s++;
    f.s = s;
    f.m = (uint32_t)((((1ull << s) - d) << 32) / d + 1);
    return f;
}

WCL_D uint32_t fdiv(uint32_t n, const FastDiv &f) { return (__umulhi(n, f.m) + n) >> f.s; }

inline uint32_t fdiv_host(uint32_t n, const FastDiv &f)
{
    return (uint32_t)((((uint64_t)n * f.m) >> 32) + n) >> f.s;
}

// ---------------------------------------------------------------------------
struct Geom {
    int L[4];        // lattice extents
    int B[4];        // tile extents (even, divide L)
    int NB[4];       // tiles per direction
    int Vh;          // sites per parity
    int Hb;          // sites per parity per tile
    int tbc;         // +1 periodic, -1 antiperiodic in t (fermion hops)
    int sl[4];       // strides of the in-tile lexicographic index
    int sb[4];       // strides of the tile index
    FastDiv dHb, dNB0, dNB1, dNB2, dBh0, dB1, dB2;
};

// Coordinates of the site with half index h and parity p.
struct Site {
    int x[4];   // global coordinates
    int l[4];   // coordinates inside the tile
    int b[4];   // tile coordinates
    int blk;    // tile index
    int lin;    // lexicographic index inside the tile
};

WCL_D Site decompose(const Geom &g, int h, int p)
{
    Site s;
    const uint32_t blk = fdiv((uint32_t)h, g.dHb);
    const uint32_t l2 = (uint32_t)h - blk * (uint32_t)g.Hb;
    uint32_t r = blk, q;
    q = fdiv(r, g.dNB0); const int b0 = (int)(r - q * g.NB[0]); r = q;
    q = fdiv(r, g.dNB1); const int b1 = (int)(r - q * g.NB[1]); r = q;
    q = fdiv(r, g.dNB2); const int b2 = (int)(r - q * g.NB[2]); const int b3 = (int)q;
    r = l2;
    q = fdiv(r, g.dBh0); const int lxh = (int)(r - q * (g.B[0] >> 1)); r = q;
    q = fdiv(r, g.dB1); const int l1 = (int)(r - q * g.B[1]); r = q;
    q = fdiv(r, g.dB2); const int l2c = (int)(r - q * g.B[2]); const int l3 = (int)q;
    const int l0 = 2 * lxh + ((p + l1 + l2c + l3) & 1);
    s.l[0] = l0; s.l[1] = l1; s.l[2] = l2c; s.l[3] = l3;
    s.b[0] = b0; s.b[1] = b1; s.b[2] = b2; s.b[3] = b3;
    s.x[0] = b0 * g.B[0] + l0;
    s.x[1] = b1 * g.B[1] + l1;
    s.x[2] = b2 * g.B[2] + l2c;
    s.x[3] = b3 * g.B[3] + l3;
    s.blk = (int)blk;
    s.lin = l0 + g.B[0] * (l1 + g.B[1] * (l2c + g.B[2] * l3));
    return s;
}

// Half index of the neighbour of s in direction mu (dir = +1 / -1); the tile
// index changes only when the step leaves the tile (wrapping the lattice).
WCL_D int neighbour(const Geom &g, const Site &s, int mu, int dir)
{
    int lin = s.lin, blk = s.blk;
    const int lc = s.l[mu] + dir;
    const int bc = s.b[mu];
    if (lc >= 0 && lc < g.B[mu]) {
        lin += dir * g.sl[mu];
    } else {
        lin -= dir * (g.B[mu] - 1) * g.sl[mu];
        const int nbc = bc + dir;
        if (nbc < 0) blk += (g.NB[mu] - 1) * g.sb[mu];
        else if (nbc >= g.NB[mu]) blk -= (g.NB[mu] - 1) * g.sb[mu];
        else blk += dir * g.sb[mu];
    }
    return blk * g.Hb + (lin >> 1);
}

// ---------------------------------------------------------------------------
// Complex arithmetic.
template <typename R>
struct cplx {
    R re, im;
};

template <typename R> WCL_HD cplx<R> cmk(R a, R b) { return cplx<R>{a, b}; }
template <typename R> WCL_HD cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> WCL_HD cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> WCL_HD cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
// Every fused multiply-add is written out (the library is built without
// implicit contraction), so a kernel's rounding is what its source says,
// whatever the surrounding code: variants of a kernel (staged or not, other
// launch shapes) give bitwise equal results.
WCL_HD float fmar(float a, float b, float c) { return fmaf(a, b, c); }
WCL_HD double fmar(double a, double b, double c) { return fma(a, b, c); }
template <typename R> WCL_HD cplx<R> operator*(cplx<R> a, cplx<R> b)
{
    return {fmar(a.re, b.re, -(a.im * b.im)), fmar(a.re, b.im, a.im * b.re)};
}
template <typename R> WCL_HD cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> WCL_HD cplx<R> conjm(cplx<R> a, cplx<R> b)  // conj(a) * b
{
    return {fmar(a.re, b.re, a.im * b.im), fmar(a.re, b.im, -(a.im * b.re))};
}
template <typename R> WCL_HD cplx<R> cfma(cplx<R> a, cplx<R> b, cplx<R> c)  // a*b + c
{
    return {fmar(a.re, b.re, fmar(-a.im, b.im, c.re)), fmar(a.re, b.im, fmar(a.im, b.re, c.im))};
}
template <typename R> WCL_HD cplx<R> cjfma(cplx<R> a, cplx<R> b, cplx<R> c)  // conj(a)*b + c
{
    return {fmar(a.re, b.re, fmar(a.im, b.im, c.re)), fmar(a.re, b.im, fmar(-a.im, b.re, c.im))};
}

// Multiplication by the unit i^code, code = 0:+1, 1:+i, 2:-1, 3:-i.
template <int CODE, typename R> WCL_D cplx<R> mul_unit(cplx<R> a)
{
    if constexpr ((CODE & 3) == 0) return a;
    else if constexpr ((CODE & 3) == 1) return {-a.im, a.re};
    else if constexpr ((CODE & 3) == 2) return {-a.re, -a.im};
    else return {a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Chiral basis: gamma_mu = [[0, G_mu], [G_mu^dag, 0]] with G_x = -i s1,
// G_y = -i s2, G_z = -i s3, G_t = 1.  Every row of G and G^dag has a single
// non-zero entry, a unit i^code:  (G psi_lo)_r = i^GC[mu][r] psi_lo[GCOL[mu][r]].
__host__ __device__ constexpr int gcol(int mu, int r) { return (mu <= 1) ? 1 - r : r; }
__host__ __device__ constexpr int gcode(int mu, int r)
{
    return mu == 0 ? 3 : mu == 1 ? (r == 0 ? 2 : 0) : mu == 2 ? (r == 0 ? 3 : 1) : 0;
}
__host__ __device__ constexpr int gdcode(int mu, int r)
{
    return mu == 0 ? 1 : mu == 1 ? (r == 0 ? 0 : 2) : mu == 2 ? (r == 0 ? 1 : 3) : 0;
}

// Half spinor for the projector (1 + S gamma_mu):  h = psi_up + S G psi_lo.
template <int MU, int S, typename R>
WCL_D void project(const cplx<R> psi[12], cplx<R> h[6])
{
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int c0 = gcol(MU, r);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cplx<R> lo = psi[(2 + c0) * 3 + c];
            cplx<R> t;
            if (r == 0) t = mul_unit<gcode(MU, 0) + (S < 0 ? 2 : 0)>(lo);
            else t = mul_unit<gcode(MU, 1) + (S < 0 ? 2 : 0)>(lo);
            h[r * 3 + c] = psi[r * 3 + c] + t;
        }
    }
}

// acc += (1 + S gamma_mu) applied to a projected, colour-rotated half spinor:
// upper += uh, lower += S G^dag uh.
template <int MU, int S, typename R>
WCL_D void accumulate(cplx<R> acc[12], const cplx<R> uh[6])
{
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int c0 = gcol(MU, r);  // G^dag has the same column pattern as G
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[r * 3 + c] = acc[r * 3 + c] + uh[r * 3 + c];
            cplx<R> t;
            if (r == 0) t = mul_unit<gdcode(MU, 0) + (S < 0 ? 2 : 0)>(uh[c0 * 3 + c]);
            else t = mul_unit<gdcode(MU, 1) + (S < 0 ? 2 : 0)>(uh[c0 * 3 + c]);
            acc[(2 + r) * 3 + c] = acc[(2 + r) * 3 + c] + t;
        }
    }
}

// ---------------------------------------------------------------------------
// Storage formats.  R12f / R12h: links stored as their first two rows (12
// reals, FP32 / FP16); the third row of an SU(3) matrix is conj(row0 x row1)
// and is rebuilt in registers.  The clover field of those tiers is FP32 /
// FP16.
struct R12f {};
struct R12h {};
template <typename S> struct Real { using T = float; };
template <> struct Real<double> { using T = double; };
template <typename S> struct ClovS { using T = S; };
template <> struct ClovS<R12f> { using T = float; };
template <> struct ClovS<R12h> { using T = __half; };

WCL_D float2 h2f2(uint32_t u)
{
    __half2 h = *reinterpret_cast<__half2 *>(&u);
    return __half22float2(h);
}
// FP32 to FP16 (round to nearest even) of values rounded to FP32 first.  The
// empty asm keeps the compiler from folding the multiply-add that produced a
// value into the conversion (one rounding straight to FP16), which it does in
// some code shapes and not in others: FP16 results would then depend on the
// code around the store.
WCL_D void fp32_as_computed(float &a, float &b) { asm("" : "+v"(a), "+v"(b)); }
WCL_D uint32_t f22h(float a, float b)
{
    fp32_as_computed(a, b);
    __half2 h = __floats2half2_rn(a, b);
    return *reinterpret_cast<uint32_t *>(&h);
}

// Every field access is a uniform base pointer plus a 32-bit byte offset
// (fields are below 4 GiB), which keeps one VGPR per address instead of two.
template <typename T>
WCL_D T ldf(const void *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
// Non-temporal variant for data read exactly once per launch (links, clover
// of the hopping kernel): keeps it from evicting reusable lines from L2.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
WCL_D T ldf_nt(const void *base, uint32_t off)
{
    const char *p = reinterpret_cast<const char *>(base) + off;
    T r;
    if constexpr (sizeof(T) == 16) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        __builtin_memcpy(&r, &v, 16);
    } else if constexpr (sizeof(T) == 8) {
        const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
        __builtin_memcpy(&r, &v, 8);
    } else {
        const unsigned int v = __builtin_nontemporal_load(reinterpret_cast<const unsigned int *>(p));
        __builtin_memcpy(&r, &v, 4);
    }
    return r;
}

template <bool NT, typename T>
WCL_D T ldx(const void *base, uint32_t off)
{
    if constexpr (NT) return ldf_nt<T>(base, off);
    else return ldf<T>(base, off);
}

template <typename T>
WCL_D void stf(void *base, uint32_t off, const T &v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

template <typename S, typename R>
WCL_D void load_spinor(const void *base, uint32_t h, uint32_t Vh, cplx<R> v[12])
{
    static_assert(!std::is_empty<S>::value, "two-row link tags are link storage only");
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t i = 0; i < 12; i++) {
            const double2 d = ldf<double2>(base, (i * Vh + h) * 16u);
            v[i] = {(R)d.x, (R)d.y};
        }
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 6; k++) {
            const float4 f = ldf<float4>(base, (k * Vh + h) * 16u);
            v[2 * k] = {(R)f.x, (R)f.y};
            v[2 * k + 1] = {(R)f.z, (R)f.w};
        }
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) {
            const uint4 u = ldf<uint4>(base, (k * Vh + h) * 16u);
            float2 a = h2f2(u.x), b = h2f2(u.y), c = h2f2(u.z), d = h2f2(u.w);
            v[4 * k + 0] = {(R)a.x, (R)a.y};
            v[4 * k + 1] = {(R)b.x, (R)b.y};
            v[4 * k + 2] = {(R)c.x, (R)c.y};
            v[4 * k + 3] = {(R)d.x, (R)d.y};
        }
    }
}

template <typename S, typename R>
WCL_D void store_spinor(void *base, uint32_t h, uint32_t Vh, const cplx<R> v[12])
{
    static_assert(!std::is_empty<S>::value, "two-row link tags are link storage only");
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t i = 0; i < 12; i++) stf(base, (i * Vh + h) * 16u, make_double2((double)v[i].re, (double)v[i].im));
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 6; k++)
            stf(base, (k * Vh + h) * 16u,
                make_float4((float)v[2 * k].re, (float)v[2 * k].im, (float)v[2 * k + 1].re, (float)v[2 * k + 1].im));
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) {
            uint4 u;
            u.x = f22h((float)v[4 * k].re, (float)v[4 * k].im);
            u.y = f22h((float)v[4 * k + 1].re, (float)v[4 * k + 1].im);
            u.z = f22h((float)v[4 * k + 2].re, (float)v[4 * k + 2].im);
            u.w = f22h((float)v[4 * k + 3].re, (float)v[4 * k + 3].im);
            stf(base, (k * Vh + h) * 16u, u);
        }
    }
}

template <typename R>
WCL_D void su3_third_row(cplx<R> u[9])
{
    // row 2 = conj(row 0 x row 1)
    const cplx<R> c0 = cfma(u[1], u[5], -(u[2] * u[4]));
    const cplx<R> c1 = cfma(u[2], u[3], -(u[0] * u[5]));
    const cplx<R> c2 = cfma(u[0], u[4], -(u[1] * u[3]));
    u[6] = {c0.re, -c0.im};
    u[7] = {c1.re, -c1.im};
    u[8] = {c2.re, -c2.im};
}

// A link as loaded (still encoded), so that a pipeline stage holds 12 (two
// rows) or 18 reals and decodes at compute time.
template <typename S> struct LinkRaw { float4 v[4]; float2 w; };
template <> struct LinkRaw<double> { double2 v[9]; };
template <> struct LinkRaw<__half> { uint4 v[2]; uint32_t w; };
template <> struct LinkRaw<R12f> { float4 v[3]; };
template <> struct LinkRaw<R12h> { uint4 v; uint2 w; };

template <typename S, bool NT = false>
WCL_D void load_link_raw(const void *base, int mu, int p, uint32_t h, uint32_t Vh, LinkRaw<S> &r)
{
    const uint32_t mp = (uint32_t)(mu * 2 + p);
    if constexpr (std::is_same<S, R12f>::value) {
        // float4 [4][2][3][Vh]: rows 0 and 1
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) r.v[k] = ldx<NT, float4>(base, ((mp * 3 + k) * Vh + h) * 16u);
    } else if constexpr (std::is_same<S, R12h>::value) {
        // 8 halves [4][2][Vh] (complex 0..3) + 4 halves [4][2][Vh] (complex 4, 5)
        r.v = ldx<NT, uint4>(base, (mp * Vh + h) * 16u);
        r.w = ldx<NT, uint2>(base, 8u * Vh * 16u + (mp * Vh + h) * 8u);
    } else if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t i = 0; i < 9; i++) r.v[i] = ldx<NT, double2>(base, ((mp * 9 + i) * Vh + h) * 16u);
    } else if constexpr (sizeof(S) == 4) {
        // float4 [4][2][4][Vh] (complex 0..7) + float2 [4][2][Vh] (complex 8)
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) r.v[k] = ldx<NT, float4>(base, ((mp * 4 + k) * Vh + h) * 16u);
        r.w = ldx<NT, float2>(base, 32u * Vh * 16u + (mp * Vh + h) * 8u);
    } else {
        // uint4 [4][2][2][Vh] (complex 0..7) + half2 [4][2][Vh] (complex 8)
#pragma unroll
        for (uint32_t k = 0; k < 2; k++) r.v[k] = ldx<NT, uint4>(base, ((mp * 2 + k) * Vh + h) * 16u);
        r.w = ldx<NT, uint32_t>(base, 16u * Vh * 16u + (mp * Vh + h) * 4u);
    }
}

// A link load that reads zero where `in` is false, without a branch: the
// field is addressed through a buffer resource of 2 GiB (every FP32 / FP16
// link field is smaller: the FP64 one is below 4 GiB), and a cut lane's
// offset is moved to 2 GiB or more, where the load reads zero and touches no
// memory.  Being unconditional, the loads also keep the compiler's wait
// counts exact in a software pipeline (a load under a branch turns each
// later wait for it into a wait for every load in flight).
WCL_D __amdgpu_buffer_rsrc_t field_rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)0x80000000u, 0x00020000);
}
template <typename T>
WCL_D T ldb(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    T r;
    if constexpr (sizeof(T) == 16) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        __builtin_memcpy(&r, &v, 16);
    } else if constexpr (sizeof(T) == 8) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        __builtin_memcpy(&r, &v, 8);
    } else {
        const unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        __builtin_memcpy(&r, &v, 4);
    }
    return r;
}

// R12f: from the per-site copy (store_link_site).
template <typename S>
WCL_D void load_link_raw_or_zero(__amdgpu_buffer_rsrc_t rs, int mu, int p, uint32_t h, bool in, uint32_t Vh,
                                 LinkRaw<S> &r)
{
    static_assert(sizeof(S) != 8, "FP64 links are not read through a 2 GiB resource");
    constexpr uint32_t OUT = 0x80000000u;
    const uint32_t mp = (uint32_t)(mu * 2 + p);
    const uint32_t o16 = in ? h * 16u : OUT, o8 = in ? h * 8u : OUT, o4 = in ? h * 4u : OUT;
    if constexpr (std::is_same<S, R12f>::value) {
        // the per-site copy (store_link_site)
        const uint32_t o48 = in ? (mp * Vh + h) * 48u : OUT;
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) r.v[k] = ldb<float4>(rs, o48 + k * 16u);
    } else if constexpr (std::is_same<S, R12h>::value) {
        r.v = ldb<uint4>(rs, mp * Vh * 16u + o16);
        r.w = ldb<uint2>(rs, 8u * Vh * 16u + mp * Vh * 8u + o8);
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) r.v[k] = ldb<float4>(rs, (mp * 4 + k) * Vh * 16u + o16);
        r.w = ldb<float2>(rs, 32u * Vh * 16u + mp * Vh * 8u + o8);
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 2; k++) r.v[k] = ldb<uint4>(rs, (mp * 2 + k) * Vh * 16u + o16);
        r.w = ldb<uint32_t>(rs, 16u * Vh * 16u + mp * Vh * 4u + o4);
    }
}

// Per-site copy of the two-row FP32 links, [mu][parity][Vh][12 reals] (48
// contiguous bytes a link): the fused Schwarz kernel gathers the links of
// scattered block sites, and one link then spans one or two cache lines
// instead of three partly used ones.
template <typename R>
WCL_D void store_link_site(void *base, int mu, int p, uint32_t h, uint32_t Vh, const cplx<R> u[9])
{
    const uint32_t mp = (uint32_t)(mu * 2 + p);
#pragma unroll
    for (uint32_t k = 0; k < 3; k++)
        stf(base, (mp * Vh + h) * 48u + k * 16u,
            make_float4((float)u[2 * k].re, (float)u[2 * k].im, (float)u[2 * k + 1].re, (float)u[2 * k + 1].im));
}

template <typename S, typename R>
WCL_D void expand_link(const LinkRaw<S> &r, cplx<R> u[9])
{
    if constexpr (std::is_same<S, R12f>::value) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            u[2 * k] = {(R)r.v[k].x, (R)r.v[k].y};
            u[2 * k + 1] = {(R)r.v[k].z, (R)r.v[k].w};
        }
        su3_third_row(u);
    } else if constexpr (std::is_same<S, R12h>::value) {
        const float2 a = h2f2(r.v.x), b = h2f2(r.v.y), c = h2f2(r.v.z), d = h2f2(r.v.w), e = h2f2(r.w.x),
                     f = h2f2(r.w.y);
        u[0] = {(R)a.x, (R)a.y}; u[1] = {(R)b.x, (R)b.y}; u[2] = {(R)c.x, (R)c.y};
        u[3] = {(R)d.x, (R)d.y}; u[4] = {(R)e.x, (R)e.y}; u[5] = {(R)f.x, (R)f.y};
        su3_third_row(u);
    } else if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (int i = 0; i < 9; i++) u[i] = {(R)r.v[i].x, (R)r.v[i].y};
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            u[2 * k] = {(R)r.v[k].x, (R)r.v[k].y};
            u[2 * k + 1] = {(R)r.v[k].z, (R)r.v[k].w};
        }
        u[8] = {(R)r.w.x, (R)r.w.y};
    } else {
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const float2 a = h2f2(r.v[k].x), b = h2f2(r.v[k].y), c = h2f2(r.v[k].z), d = h2f2(r.v[k].w);
            u[4 * k + 0] = {(R)a.x, (R)a.y};
            u[4 * k + 1] = {(R)b.x, (R)b.y};
            u[4 * k + 2] = {(R)c.x, (R)c.y};
            u[4 * k + 3] = {(R)d.x, (R)d.y};
        }
        const float2 f = h2f2(r.w);
        u[8] = {(R)f.x, (R)f.y};
    }
}

// Link U_mu at (parity p, half index h): 9 complex, row-major.
template <typename S, typename R, bool NT = false>
WCL_D void load_link(const void *base, int mu, int p, uint32_t h, uint32_t Vh, cplx<R> u[9])
{
    LinkRaw<S> r;
    load_link_raw<S, NT>(base, mu, p, h, Vh, r);
    expand_link<S, R>(r, u);
}

template <typename S, typename R>
WCL_D void store_link(void *base, int mu, int p, uint32_t h, uint32_t Vh, const cplx<R> u[9])
{
    const uint32_t mp = (uint32_t)(mu * 2 + p);
    if constexpr (std::is_same<S, R12f>::value) {
#pragma unroll
        for (uint32_t k = 0; k < 3; k++)
            stf(base, ((mp * 3 + k) * Vh + h) * 16u,
                make_float4((float)u[2 * k].re, (float)u[2 * k].im, (float)u[2 * k + 1].re, (float)u[2 * k + 1].im));
    } else if constexpr (std::is_same<S, R12h>::value) {
        uint4 w;
        w.x = f22h((float)u[0].re, (float)u[0].im);
        w.y = f22h((float)u[1].re, (float)u[1].im);
        w.z = f22h((float)u[2].re, (float)u[2].im);
        w.w = f22h((float)u[3].re, (float)u[3].im);
        stf(base, (mp * Vh + h) * 16u, w);
        uint2 v;
        v.x = f22h((float)u[4].re, (float)u[4].im);
        v.y = f22h((float)u[5].re, (float)u[5].im);
        stf(base, 8u * Vh * 16u + (mp * Vh + h) * 8u, v);
    } else if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t i = 0; i < 9; i++)
            stf(base, ((mp * 9 + i) * Vh + h) * 16u, make_double2((double)u[i].re, (double)u[i].im));
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 4; k++)
            stf(base, ((mp * 4 + k) * Vh + h) * 16u,
                make_float4((float)u[2 * k].re, (float)u[2 * k].im, (float)u[2 * k + 1].re, (float)u[2 * k + 1].im));
        stf(base, 32u * Vh * 16u + (mp * Vh + h) * 8u, make_float2((float)u[8].re, (float)u[8].im));
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 2; k++) {
            uint4 w;
            w.x = f22h((float)u[4 * k].re, (float)u[4 * k].im);
            w.y = f22h((float)u[4 * k + 1].re, (float)u[4 * k + 1].im);
            w.z = f22h((float)u[4 * k + 2].re, (float)u[4 * k + 2].im);
            w.w = f22h((float)u[4 * k + 3].re, (float)u[4 * k + 3].im);
            stf(base, ((mp * 2 + k) * Vh + h) * 16u, w);
        }
        stf(base, 16u * Vh * 16u + (mp * Vh + h) * 4u, f22h((float)u[8].re, (float)u[8].im));
    }
}

// Bytes of one link field (both parities, 4 directions) in storage S.
WCL_HD size_t link_bytes(int S_size, size_t Vh)
{
    return S_size == 8 ? 72 * 16 * Vh : S_size == 4 ? (32 * 16 + 8 * 8) * Vh : (16 * 16 + 8 * 4) * Vh;
}
WCL_HD size_t spinor_bytes(int S_size, size_t Vh) { return (S_size == 8 ? 192 : S_size == 4 ? 96 : 48) * Vh; }
WCL_HD size_t clover_bytes(int S_size, size_t Vh) { return 2 * (S_size == 8 ? 576 : S_size == 4 ? 288 : 144) * Vh; }

// Clover site (72 reals) at (parity p, h).
template <typename S, typename R, bool NT = false>
WCL_D void load_clover(const void *base, int p, uint32_t h, uint32_t Vh, R c[72])
{
    static_assert(!std::is_empty<S>::value, "two-row link tags are link storage only");
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t k = 0; k < 36; k++) {
            const double2 d = ldx<NT, double2>(base, (((uint32_t)p * 36 + k) * Vh + h) * 16u);
            c[2 * k] = (R)d.x;
            c[2 * k + 1] = (R)d.y;
        }
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 18; k++) {
            const float4 f = ldx<NT, float4>(base, (((uint32_t)p * 18 + k) * Vh + h) * 16u);
            c[4 * k] = f.x; c[4 * k + 1] = f.y; c[4 * k + 2] = f.z; c[4 * k + 3] = f.w;
        }
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 9; k++) {
            const uint4 w = ldx<NT, uint4>(base, (((uint32_t)p * 9 + k) * Vh + h) * 16u);
            float2 a = h2f2(w.x), b = h2f2(w.y), cc = h2f2(w.z), d = h2f2(w.w);
            c[8 * k + 0] = a.x; c[8 * k + 1] = a.y; c[8 * k + 2] = b.x; c[8 * k + 3] = b.y;
            c[8 * k + 4] = cc.x; c[8 * k + 5] = cc.y; c[8 * k + 6] = d.x; c[8 * k + 7] = d.y;
        }
    }
}

template <typename S>
WCL_D void store_clover(void *base, int p, uint32_t h, uint32_t Vh, const double c[72])
{
    static_assert(!std::is_empty<S>::value, "two-row link tags are link storage only");
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t k = 0; k < 36; k++)
            stf(base, (((uint32_t)p * 36 + k) * Vh + h) * 16u, make_double2(c[2 * k], c[2 * k + 1]));
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 18; k++)
            stf(base, (((uint32_t)p * 18 + k) * Vh + h) * 16u,
                make_float4((float)c[4 * k], (float)c[4 * k + 1], (float)c[4 * k + 2], (float)c[4 * k + 3]));
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 9; k++) {
            uint4 w;
            w.x = f22h((float)c[8 * k], (float)c[8 * k + 1]);
            w.y = f22h((float)c[8 * k + 2], (float)c[8 * k + 3]);
            w.z = f22h((float)c[8 * k + 4], (float)c[8 * k + 5]);
            w.w = f22h((float)c[8 * k + 6], (float)c[8 * k + 7]);
            stf(base, (((uint32_t)p * 9 + k) * Vh + h) * 16u, w);
        }
    }
}

// One chirality block (36 reals) of a clover site: half 0 = spins 0,1,
// half 1 = spins 2,3.  ClovHalfRaw holds it as loaded (decoded later).
template <typename S> struct ClovHalfRaw { float4 v[9]; };
template <> struct ClovHalfRaw<double> { double2 v[18]; };
template <> struct ClovHalfRaw<__half> { uint4 v[5]; };

template <typename S>
WCL_D void load_clover_half_raw(const void *base, int p, uint32_t h, uint32_t Vh, int half, ClovHalfRaw<S> &r)
{
    static_assert(!std::is_empty<S>::value, "two-row link tags are link storage only");
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t k = 0; k < 18; k++) r.v[k] = ldf<double2>(base, (((uint32_t)p * 36 + 18 * half + k) * Vh + h) * 16u);
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 9; k++) r.v[k] = ldf<float4>(base, (((uint32_t)p * 18 + 9 * half + k) * Vh + h) * 16u);
    } else {
        // 36 halves starting at half 36*half: uint4 words w0 .. w0+4 (8 halves each)
        const uint32_t w0 = half ? 4u : 0u;
#pragma unroll
        for (uint32_t k = 0; k < 5; k++) r.v[k] = ldf<uint4>(base, (((uint32_t)p * 9 + w0 + k) * Vh + h) * 16u);
    }
}

template <typename S, typename R>
WCL_D void expand_clover_half(const ClovHalfRaw<S> &r, int half, R c[36])
{
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (int k = 0; k < 18; k++) {
            c[2 * k] = (R)r.v[k].x;
            c[2 * k + 1] = (R)r.v[k].y;
        }
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            c[4 * k] = r.v[k].x; c[4 * k + 1] = r.v[k].y; c[4 * k + 2] = r.v[k].z; c[4 * k + 3] = r.v[k].w;
        }
    } else {
        float t[40];
#pragma unroll
        for (int k = 0; k < 5; k++) {
            float2 a = h2f2(r.v[k].x), b = h2f2(r.v[k].y), cc = h2f2(r.v[k].z), d = h2f2(r.v[k].w);
            t[8 * k + 0] = a.x; t[8 * k + 1] = a.y; t[8 * k + 2] = b.x; t[8 * k + 3] = b.y;
            t[8 * k + 4] = cc.x; t[8 * k + 5] = cc.y; t[8 * k + 6] = d.x; t[8 * k + 7] = d.y;
        }
        const int off = half ? 4 : 0;
#pragma unroll
        for (int k = 0; k < 36; k++) c[k] = (R)t[off + k];
    }
}

template <typename S, typename R>
WCL_D void load_clover_half(const void *base, int p, uint32_t h, uint32_t Vh, int half, R c[36])
{
    ClovHalfRaw<S> r;
    load_clover_half_raw<S>(base, p, h, Vh, half, r);
    expand_clover_half<S, R>(r, half, c);
}

template <typename R>
WCL_D void clover_mul_half(const R blk[36], const cplx<R> x[6], cplx<R> y[6])
{
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = blk[i] * x[i];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            const cplx<R> a = {blk[6 + 2 * k], blk[7 + 2 * k]};
            y[i] = cfma(a, x[j], y[i]);
            y[j] = cjfma(a, x[i], y[j]);
            k++;
        }
}

// out = A v for a packed Hermitian clover site (two 6x6 blocks): 504 flop.
template <typename R>
WCL_D void clover_mul(const R c[72], const cplx<R> v[12], cplx<R> out[12])
{
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const R *blk = c + 36 * b;
        const cplx<R> *x = v + 6 * b;
        cplx<R> *y = out + 6 * b;
#pragma unroll
        for (int i = 0; i < 6; i++) y[i] = blk[i] * x[i];
        int k = 0;
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = i + 1; j < 6; j++) {
                const cplx<R> a = {blk[6 + 2 * k], blk[7 + 2 * k]};
                y[i] = cfma(a, x[j], y[i]);
                y[j] = cjfma(a, x[i], y[j]);
                k++;
            }
    }
}

// SU(3) (or any 3x3) times the two colour vectors of a half spinor.
template <typename R>
WCL_D void su3_mul(const cplx<R> u[9], const cplx<R> h[6], cplx<R> o[6])
{
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cplx<R> acc = u[a * 3] * h[s * 3];
            acc = cfma(u[a * 3 + 1], h[s * 3 + 1], acc);
            acc = cfma(u[a * 3 + 2], h[s * 3 + 2], acc);
            o[s * 3 + a] = acc;
        }
}

template <typename R>
WCL_D void su3_dag_mul(const cplx<R> u[9], const cplx<R> h[6], cplx<R> o[6])
{
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cplx<R> acc = conjm(u[a], h[s * 3]);
            acc = cjfma(u[3 + a], h[s * 3 + 1], acc);
            acc = cjfma(u[6 + a], h[s * 3 + 2], acc);
            o[s * 3 + a] = acc;
        }
}

// The thread's index in its workgroup as a value the compiler cannot prove
// loop-invariant: per-thread arithmetic of a code path that runs inside a
// long kernel loop (the persistent solver's phases) stays in that path
// instead of being hoisted to the kernel entry and held in registers.
WCL_D unsigned tid_here()
{
    unsigned t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// XCD-aware workgroup order: consecutive logical tiles land on one XCD
// (workgroups are dealt round-robin over the 8 XCDs).
WCL_D int xcd_block(int bid, int nblk)
{
    const int per = nblk >> 3;
    if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
    return bid;
}

}  // namespace wcl
