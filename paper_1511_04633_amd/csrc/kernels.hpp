// kernels.hpp -- HIP kernels of the double-MRT cavity step for gfx950.
//
// Data layout in HBM: two lattices (ping-pong).  Nodes are numbered
// c = x + n*(y + n*z), x fastest.  A lattice is a sequence of slabs of 2^L
// consecutive nodes; a slab holds 19 D3Q19 segments of 2^L flow elements
// followed by 7 D3Q7 segments of 2^L energy elements (segment i holds
// population i of the slab's nodes, in node order).  A wavefront therefore
// reads and writes 64 consecutive elements per population, and the 26
// population streams of a block of rows lie within one slab (a few hundred
// KB) instead of 26 planes n^3 elements apart, which measured about 6%
// faster on the pull pattern than whole-lattice planes.  L is fixed per
// storage format so that a flow segment is 8 KB.
//
// What a lattice holds: the post-collision populations f*(t-1), g*(t-1).
// The step kernel gathers ("pulls") them from the upstream neighbours, which
// is streaming (Eq. 14, Eq. 29) together with the wall conditions, then
// collides in registers and writes f*(t), g*(t) at the node itself (aligned
// stores).  Reads of the state at time t (fields, Nu, populations) perform
// the same pull without colliding.  Initialising a state S_0 therefore means
// writing the unique post-collision set whose pull gives S_0 ("unstream").
//
// Wall conditions in pull form (walls half way between nodes, at rest):
//   D3Q19: f_i(x) = f*_ibar(x) when x - e_i is outside (bounce-back, Eq. 8);
//   D3Q7 : g_i(x) = -g*_ibar(x) + 2 w_T,i theta_W on a Dirichlet wall,
//          g_i(x) =  g*_ibar(x) on an adiabatic wall.
// Each D3Q7 link crosses a single wall, so edges and corners need no rule.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "collide.hpp"

namespace lbmx {

// ------------------------------------------------------------------ storage
// Codec<S>: how one population is held in HBM.  Flow populations are stored
// as offsets df = f - w_i, energy populations as g; the 16-bit formats store
// df / w_i and g / w_T,i (the population relative to its weight), which keeps
// every direction's stored value O(u) or O(theta).  `Raw` is the bit
// container: loads return it and dec() reinterprets its bits; `inv_w` is the
// exact reciprocal of the weight (3, 18, 36; 4, 8), so encoding multiplies
// instead of dividing.
template <typename S>
struct Codec;

template <>
struct Codec<double> {
    using Raw = double;
    template <typename T> static __device__ __forceinline__ T dec(Raw v, T) { return T(v); }
    template <typename T> static __device__ __forceinline__ Raw enc(T v, T) { return double(v); }
};

template <>
struct Codec<float> {
    using Raw = float;
    template <typename T> static __device__ __forceinline__ T dec(Raw v, T) { return T(v); }
    template <typename T> static __device__ __forceinline__ Raw enc(T v, T) { return float(v); }
};

template <>
struct Codec<__half> {
    using Raw = unsigned short;
    template <typename T> static __device__ __forceinline__ T dec(Raw v, T w)
    {
        return T(__half2float(__ushort_as_half(v))) * w;
    }
    template <typename T> static __device__ __forceinline__ Raw enc(T v, T inv_w)
    {
        return __half_as_ushort(__float2half_rn(float(v * inv_w)));
    }
};

template <>
struct Codec<__hip_bfloat16> {
    using Raw = unsigned short;
    template <typename T> static __device__ __forceinline__ T dec(Raw v, T w)
    {
        return T(__bfloat162float(__ushort_as_bfloat16(v))) * w;
    }
    template <typename T> static __device__ __forceinline__ Raw enc(T v, T inv_w)
    {
        return __bfloat16_as_ushort(__float2bfloat16(float(v * inv_w)));
    }
};

// log2 of the nodes per slab for a flow element of `flow_bytes` bytes:
// 8 KB flow segments (2^10 FP64, 2^11 FP32, 2^12 16-bit elements).
__host__ __device__ constexpr int slab_shift_for(size_t flow_bytes)
{
    return flow_bytes >= 8 ? 10 : (flow_bytes == 4 ? 11 : 12);
}

// Fixed-point energy storage: g_i / (w_T,i Theta) as a signed 16-bit integer
// in units of 2^-15 (range +-1).  Theta is the power of two at or above
// 2 max(|theta_hot|, |theta_cold|) (1 for the walls at +-1/2), so that
// |g_i / w_T,i| = |theta (1 + 4 e_i.u)| + non-equilibrium part stays below
// Theta; the spacing is then 3.1e-5 Theta, uniform (FP16's is 1.2e-4 to 2.4e-4
// over the |g/w_T| = 0.25 .. 1 where the temperature signal lives).
// The step kernels round stochastically (enc_r): up with probability equal to
// the fraction below, so that a change smaller than one spacing per step is
// kept on average instead of being rounded away every step (the slow thermal
// drift would otherwise stall: with rounding to nearest a 2^-14 code's Nu
// error at 64^3, Ra 1e6 was 4.3e-3, with stochastic rounding 1.5e-5; 8
// random bits instead of 16 left a 3.6e-4 bias at steady state).
// Initialisation rounds to nearest (enc).  The weight arguments carry Theta
// (w_T,i Theta to decode, 1/(w_T,i Theta) to encode; exact, Theta being a
// power of two).  Finite values saturate at +-32767; -32768 encodes NaN, so
// that a diverging run still reports non-finite values.
struct Fix16 {
    short bits;
};

template <>
struct Codec<Fix16> {
    using Raw = unsigned short;
    template <typename T> static __device__ __forceinline__ T dec(Raw v, T w)
    {
        const short q = short(v);
        return q == -32768 ? T(NAN) : T(q) * (w * T(1.0 / 32768.0));
    }
    static __device__ __forceinline__ Raw pack(float q)
    {
        return Raw(short(fminf(fmaxf(q, -32767.0f), 32767.0f)));
    }
    template <typename T> static __device__ __forceinline__ Raw enc(T v, T inv_w)
    {
        const float x = float(v * inv_w) * 32768.0f;
        return x == x ? pack(rintf(x)) : Raw(0x8000);
    }
    // u16: 16 uniformly random bits, u = u16 / 2^16 in [0, 1).  Rounds up when
    // u < x - floor(x), i.e. with probability frac(x) (to 2^-16).  Every
    // operation here is exact (scaling by powers of two, floor, the
    // difference of nearby floats), so the result does not depend on how the
    // compiler contracts the arithmetic around it; floor(x + u) would round
    // the sum to the spacing of x (2^-9 at |x| = 2^14) and bias the rounding.
    template <typename T> static __device__ __forceinline__ Raw enc_r(T v, T inv_w, uint32_t u16)
    {
        const float x = float(v * inv_w) * 32768.0f;
        if (!(x == x))
            return Raw(0x8000);
        const float fl = floorf(x);
        const float u = float(u16) * (1.0f / 65536.0f);
        return pack(u < x - fl ? fl + 1.0f : fl);
    }
};

// Random bits for the stochastic rounding of node c's energy populations at
// step t: the MurmurHash3 finaliser (multiply-xorshift) of a combination of
// the two counters gives the first 32-bit word, xorshift32 (Marsaglia) the
// next three; each word serves two populations, 16 bits each.
// Deterministic: a run repeats exactly.
struct RoundBits {
    uint32_t w[4];
    __device__ __forceinline__ RoundBits(uint32_t c, uint32_t t)
    {
        uint32_t h = c * 0x9E3779B1u + t * 0xC2B2AE3Du;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        h |= 1u;  // xorshift needs a nonzero state
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[k] = h;
            h ^= h << 13;
            h ^= h >> 17;
            h ^= h << 5;
        }
    }
    __device__ __forceinline__ uint32_t u16(int i) const
    {
        return (i & 1) ? (w[i >> 1] >> 16) : (w[i >> 1] & 0xffffu);
    }
};

// Element types of the flow (SF) and energy (SG) segments; T is the
// arithmetic type of the collision (FP64 only when both are FP64).
template <typename SF, typename SG>
struct Store {
    using F = SF;
    using G = SG;
    // the energy codec's weights carry the temperature scale Theta
    static constexpr bool kScaledG = std::is_same<SG, Fix16>::value;
    static constexpr int kSlabShift = slab_shift_for(sizeof(SF));
    using T = typename std::conditional<std::is_same<SF, double>::value &&
                                            std::is_same<SG, double>::value,
                                        double, float>::type;
};

// ---------------------------------------------------------- lattice tables
// D3Q19 (Eq. 12) and D3Q7 (Eq. 28) in the paper's order, 0-based.
__device__ __forceinline__ constexpr int ex19(int i)
{
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__device__ __forceinline__ constexpr int ey19(int i)
{
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__device__ __forceinline__ constexpr int ez19(int i)
{
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
}
__device__ __forceinline__ constexpr int opp19(int i)
{
    constexpr int v[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[i];
}
// Eq. (18) and Eq. (31), with exact reciprocals.
__device__ __forceinline__ constexpr double w19(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__device__ __forceinline__ constexpr double w7(int i) { return i == 0 ? 0.25 : 0.125; }
__device__ __forceinline__ constexpr double inv_w19(int i) { return i == 0 ? 3.0 : (i < 7 ? 18.0 : 36.0); }
__device__ __forceinline__ constexpr double inv_w7(int i) { return i == 0 ? 4.0 : 8.0; }

// ---------------------------------------------------------------- arguments
template <typename T>
struct Geometry {
    int n;
    int wall_type;     // 1, 2, 3
    T theta_hot, theta_cold;
    uint32_t step;     // time step being written (stochastic-rounding stream)
    T escale;          // Theta of the fixed-point energy code (1 otherwise)
    T inv_escale;      // 1 / Theta (exact: Theta is a power of two)
};

// theta on a linear wall (Eqs. 9-10) at node height y: the crossing point of
// an x or z link has the node's y = j + 1/2.
template <typename T>
__device__ __forceinline__ T theta_linear(const Geometry<T> &geo, int y)
{
    return geo.theta_hot + (geo.theta_cold - geo.theta_hot) * (T(y) + T(0.5)) / T(geo.n);
}

// Dirichlet flags of the x and z walls for the three cavity types.
__device__ __forceinline__ bool x_wall_dirichlet(int wall_type) { return wall_type != 1; }
__device__ __forceinline__ bool z_wall_dirichlet(int wall_type) { return wall_type == 2; }

// ----------------------------------------------------------------- access
// Byte offsets are 32-bit when a whole lattice spans less than 4 GiB: a load
// is then a uniform 64-bit base plus a 32-bit per-lane offset (one VALU add
// per population instead of 64-bit address arithmetic); larger lattices use
// 64-bit offsets.  Stores are non-temporal: the written lattice is read back
// only in the next step, long after it has left the caches.
template <bool kOff32>
struct Access {
    using I = typename std::conditional<kOff32, uint32_t, size_t>::type;
    // Lattices live in device global memory; saying so lets pointers read from
    // a table (batch kernel) use global rather than flat instructions.
    template <typename S>
    using gptr = __attribute__((address_space(1))) S *;
    // Loads return the storage bits (Codec<S>::Raw); Codec<S>::dec converts.
    // 8-byte populations (FP64 storage) are read non-temporally as well
    // (measured 2.5 % faster at 256^3); narrower ones are not (slower: a
    // wavefront's x-shifted reads share cache lines with its neighbours').
    template <typename S>
    static __device__ __forceinline__ typename Codec<S>::Raw ld(const char *base, I byte)
    {
        using R = typename Codec<S>::Raw;
        if constexpr (sizeof(R) == 8)
            return __builtin_nontemporal_load((gptr<const R>)((gptr<const char>)base + byte));
        else
            return *(gptr<const R>)((gptr<const char>)base + byte);
    }
    template <typename S>
    static __device__ __forceinline__ void st(char *base, I byte, typename Codec<S>::Raw v)
    {
        using R = typename Codec<S>::Raw;
        __builtin_nontemporal_store(v, (gptr<R>)((gptr<char>)base + byte));
    }
};

// Byte offsets of population i of node c inside a lattice (slab layout
// above): slab (c >> L) * slab_bytes + segment i + slot (c mod 2^L), written
// as c * b + (c >> L) * (slab_bytes - segment_bytes) + i * segment_bytes.
// Every term is below the lattice size, so 32-bit offsets cannot wrap.
template <class St, bool kOff32>
struct Lat {
    using I = typename Access<kOff32>::I;
    static constexpr int L = St::kSlabShift;
    static constexpr I bF = I(sizeof(typename St::F)), bG = I(sizeof(typename St::G));
    static constexpr I segF = bF << L, segG = bG << L;
    static constexpr I slab = 19 * segF + 7 * segG;
    static __device__ __forceinline__ I f(I c, int i)
    {
        return c * bF + (c >> L) * (slab - segF) + I(i) * segF;
    }
    static __device__ __forceinline__ I g(I c, int i)
    {
        return c * bG + (c >> L) * (slab - segG) + 19 * segF + I(i) * segG;
    }
};

// ------------------------------------------------------------------- pull
// Gather the populations of node (x, y, z) at time t from the post-collision
// lattice `src` (time t-1): streaming plus wall conditions.
template <class St, bool kOff32>
__device__ __forceinline__ void pull(const char *__restrict__ src,
                                     const Geometry<typename St::T> &geo, int x, int y, int z,
                                     typename St::T f[19], typename St::T g[7])
{
    using T = typename St::T;
    using SF = typename St::F;
    using SG = typename St::G;
    using A = Access<kOff32>;
    using Lt = Lat<St, kOff32>;
    using I = typename A::I;
    const int n = geo.n;
    const I idx = I(x) + I(n) * (I(y) + I(n) * I(z));
    const bool xl = x == 0, xh = x == n - 1;
    const bool yl = y == 0, yh = y == n - 1;
    const bool zl = z == 0, zh = z == n - 1;
    const I sy = I(n), sz = I(n) * I(n);

#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int ex = ex19(i), ey = ey19(i), ez = ez19(i);
        const bool out = (ex > 0 && xl) || (ex < 0 && xh) || (ey > 0 && yl) || (ey < 0 && yh) ||
                         (ez > 0 && zl) || (ez < 0 && zh);
        // upstream node x - e_i (unsigned wrap-around arithmetic is exact here;
        // a wrapped value only occurs where `out` discards it)
        const I up = idx - I(ex) - I(ey) * sy - I(ez) * sz;
        // Inside: f*_i(x - e_i).  Outside: f*_ibar(x) reflected at the wall.
        const I e = out ? Lt::f(idx, opp19(i)) : Lt::f(up, i);
        f[i] = Codec<SF>::dec(A::template ld<SF>(src, e), T(w19(i)));
    }

    const T two_w = T(0.25);  // 2 w_T,i for the moving directions
    const T th_lin = theta_linear(geo, y);
    const bool xd = x_wall_dirichlet(geo.wall_type);
    const bool zd = z_wall_dirichlet(geo.wall_type);
    const T es = St::kScaledG ? geo.escale : T(1);
    const T wg = T(w7(1)) * es;
    auto ldg = [&](I e) { return Codec<SG>::dec(A::template ld<SG>(src, e), wg); };
    g[0] = Codec<SG>::dec(A::template ld<SG>(src, Lt::g(idx, 0)), T(w7(0)) * es);
    {   // +x from x-1 | wall x = 0
        const T v = ldg(xl ? Lt::g(idx, 2) : Lt::g(idx - 1, 1));
        g[1] = xl ? (xd ? two_w * th_lin - v : v) : v;
    }
    {   // -x from x+1 | wall x = H
        const T v = ldg(xh ? Lt::g(idx, 1) : Lt::g(idx + 1, 2));
        g[2] = xh ? (xd ? two_w * th_lin - v : v) : v;
    }
    {   // +y from y-1 | hot wall y = 0 (Eq. 6)
        const T v = ldg(yl ? Lt::g(idx, 4) : Lt::g(idx - sy, 3));
        g[3] = yl ? two_w * geo.theta_hot - v : v;
    }
    {   // -y from y+1 | cold wall y = H (Eq. 7)
        const T v = ldg(yh ? Lt::g(idx, 3) : Lt::g(idx + sy, 4));
        g[4] = yh ? two_w * geo.theta_cold - v : v;
    }
    {   // +z from z-1 | wall z = 0
        const T v = ldg(zl ? Lt::g(idx, 6) : Lt::g(idx - sz, 5));
        g[5] = zl ? (zd ? two_w * th_lin - v : v) : v;
    }
    {   // -z from z+1 | wall z = H
        const T v = ldg(zh ? Lt::g(idx, 5) : Lt::g(idx + sz, 6));
        g[6] = zh ? (zd ? two_w * th_lin - v : v) : v;
    }
}

// Write node c's 26 populations (post-collision values of step `step`).
template <class St, bool kOff32>
__device__ __forceinline__ void put(char *__restrict__ dst, size_t node, uint32_t step,
                                    const typename St::T f[19], const typename St::T g[7],
                                    typename St::T inv_es)
{
    using T = typename St::T;
    using SF = typename St::F;
    using SG = typename St::G;
    using A = Access<kOff32>;
    using Lt = Lat<St, kOff32>;
    using I = typename A::I;
    const I c = I(node);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        A::template st<SF>(dst, Lt::f(c, i), Codec<SF>::enc(f[i], T(inv_w19(i))));
    if constexpr (std::is_same<SG, Fix16>::value) {
        const RoundBits rb(uint32_t(node), step);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            A::template st<SG>(dst, Lt::g(c, i),
                               Codec<SG>::enc_r(g[i], T(inv_w7(i)) * inv_es, rb.u16(i)));
    } else {
#pragma unroll
        for (int i = 0; i < 7; ++i)
            A::template st<SG>(dst, Lt::g(c, i), Codec<SG>::enc(g[i], T(inv_w7(i))));
    }
}

// -------------------------------------------------------------- step kernel
// One thread per node; block (bx, by) over (x, y), grid.z = z.  kForce is
// the force model (LBMX_FORCE_*).
template <class St, bool kOff32, int kForce>
__global__ __launch_bounds__(1024) void k_step(const char *__restrict__ src, char *__restrict__ dst,
                                               Geometry<typename St::T> geo,
                                               Rates<typename St::T> rates)
{
    using T = typename St::T;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= geo.n || y >= geo.n)
        return;
    T f[19], g[7];
    pull<St, kOff32>(src, geo, x, y, z, f, g);
    collide<T, kForce>(f, g, rates);
    put<St, kOff32>(dst, size_t(x) + size_t(geo.n) * (size_t(y) + size_t(geo.n) * z), geo.step, f, g,
                    geo.inv_escale);
}

// --------------------------------------------------------- state sources
// Pre-collision populations of an initial state S_0, node by node, as
// offsets (flow) and plain values (energy), in double precision.
struct SourceRest {            // f = w_i, g = w_T,i theta0
    const double *theta0;      // n^3, may be null (theta 0)
    __device__ double f(int, int) const { return 0.0; }
    __device__ double g(int i, int c) const { return theta0 ? w7(i) * theta0[c] : 0.0; }
};

// Some of the 26 population arrays of a state (numbered 0..18 flow, 19..25
// energy), each n^3 doubles: population p sits at buf + slot[p] * cells
// (slot -1: not staged).  Unstreaming population i at a node needs only
// S_i and S_ibar, so a transfer can stage the populations in opposite pairs
// and write those pairs, pass after pass, through a buffer of a few
// populations.
struct SourcePops {
    const double *buf;
    size_t cells;
    signed char slot[26];
    __device__ double f(int i, int c) const
    {
        return buf[(size_t)slot[i] * cells + c] - w19(i);
    }
    __device__ double g(int i, int c) const { return buf[(size_t)slot[19 + i] * cells + c]; }
};

// Velocity / temperature (and optionally density) fields sampled
// trilinearly from a node-centred src_n^3 grid of element type E (FP32
// fields from a caller or a network, FP64 fields of another cavity):
// f = f^eq(rho, u) (Eq. 17; rho = 1 without a density field, otherwise
// 1 + (rho_src - 1) vscale^2) and
// g = w_T theta (1 + 4 e.u), whose moments are n^eq of Eq. (33).  The
// sampled velocities are multiplied by vscale (1 keeps them bitwise).
template <class E>
struct SourceFields {
    const E *u, *v, *w, *th;
    int src_n, n;
    E vscale;
    const E *rho;  // density field, or null for rho = 1
    __device__ E sample(const E *a, int x, int y, int z) const
    {
        const E s = E(src_n) / E(n);
        E p[3] = {(x + E(0.5)) * s - E(0.5), (y + E(0.5)) * s - E(0.5), (z + E(0.5)) * s - E(0.5)};
        int i0[3];
        E fr[3];
        for (int d = 0; d < 3; ++d) {
            E q = fmin(fmax(p[d], E(0)), E(src_n - 1));
            int k = min(int(floor(q)), src_n - 2 < 0 ? 0 : src_n - 2);
            i0[d] = k;
            fr[d] = q - E(k);
        }
        auto at = [&](int dx, int dy, int dz) {
            int xx = min(i0[0] + dx, src_n - 1), yy = min(i0[1] + dy, src_n - 1),
                zz = min(i0[2] + dz, src_n - 1);
            return a[xx + (size_t)src_n * (yy + (size_t)src_n * zz)];
        };
        E c00 = at(0, 0, 0) * (1 - fr[0]) + at(1, 0, 0) * fr[0];
        E c10 = at(0, 1, 0) * (1 - fr[0]) + at(1, 1, 0) * fr[0];
        E c01 = at(0, 0, 1) * (1 - fr[0]) + at(1, 0, 1) * fr[0];
        E c11 = at(0, 1, 1) * (1 - fr[0]) + at(1, 1, 1) * fr[0];
        E c0 = c00 * (1 - fr[1]) + c10 * fr[1];
        E c1 = c01 * (1 - fr[1]) + c11 * fr[1];
        return c0 * (1 - fr[2]) + c1 * fr[2];
    }
    __device__ void node(int c, double *vel, double &theta) const
    {
        int x = c % n, y = (c / n) % n, z = c / (n * n);
        vel[0] = sample(u, x, y, z) * vscale;
        vel[1] = sample(v, x, y, z) * vscale;
        vel[2] = sample(w, x, y, z) * vscale;
        theta = sample(th, x, y, z);
    }
    __device__ double f(int i, int c) const
    {
        double vel[3], t;
        node(c, vel, t);
        const int e[3] = {ex19(i), ey19(i), ez19(i)};
        double eu = e[0] * vel[0] + e[1] * vel[1] + e[2] * vel[2];
        double uu = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
        if (!rho)
            return w19(i) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        // rho - 1 scales with u_c^2 (hydrostatic and dynamic pressure), as u with u_c
        const int x = c % n, y = (c / n) % n, z = c / (n * n);
        const double dr = (double(sample(rho, x, y, z)) - 1.0) * double(vscale) * double(vscale);
        return w19(i) * (dr + (1.0 + dr) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
    __device__ double g(int i, int c) const
    {
        double vel[3], t;
        node(c, vel, t);
        const int e[3] = {i == 1 ? 1 : (i == 2 ? -1 : 0), i == 3 ? 1 : (i == 4 ? -1 : 0),
                          i == 5 ? 1 : (i == 6 ? -1 : 0)};
        return w7(i) * t * (1.0 + 4.0 * (e[0] * vel[0] + e[1] * vel[1] + e[2] * vel[2]));
    }
};

// Fields combined from two node-centred grids (FP64 fields of two other
// cavities): u = wa u_a + wb u_b, theta = wa theta_a + wb theta_b and
// rho - 1 = wa (rho_a - 1) + wb (rho_b - 1), each sampled trilinearly as by
// SourceFields (velocities scaled by its vscale, density variations by
// vscale^2); f = f^eq(rho, u) (Eq. 17) and g = w_T theta (1 + 4 e.u).
struct SourceTwoFields {
    SourceFields<double> a, b;  // with density fields
    double wa, wb;
    __device__ void node(int c, double *vel, double &theta) const
    {
        double va[3], vb[3], ta, tb;
        a.node(c, va, ta);
        b.node(c, vb, tb);
        for (int d = 0; d < 3; ++d)
            vel[d] = wa * va[d] + wb * vb[d];
        theta = wa * ta + wb * tb;
    }
    __device__ double f(int i, int c) const
    {
        double vel[3], t;
        node(c, vel, t);
        const double eu = ex19(i) * vel[0] + ey19(i) * vel[1] + ez19(i) * vel[2];
        const double uu = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
        const int x = c % a.n, y = (c / a.n) % a.n, z = c / (a.n * a.n);
        const double dr = wa * (a.sample(a.rho, x, y, z) - 1.0) * a.vscale * a.vscale +
                          wb * (b.sample(b.rho, x, y, z) - 1.0) * b.vscale * b.vscale;
        return w19(i) * (dr + (1.0 + dr) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
    __device__ double g(int i, int c) const
    {
        double vel[3], t;
        node(c, vel, t);
        const int e[3] = {i == 1 ? 1 : (i == 2 ? -1 : 0), i == 3 ? 1 : (i == 4 ? -1 : 0),
                          i == 5 ? 1 : (i == 6 ? -1 : 0)};
        return w7(i) * t * (1.0 + 4.0 * (e[0] * vel[0] + e[1] * vel[1] + e[2] * vel[2]));
    }
};

// "Unstream": write the post-collision lattice P whose pull reproduces S.
// For population i at node y: if y + e_i is inside, P_i(y) = S_i(y + e_i);
// otherwise P_i(y) is the value that the wall turns into S_ibar(y).  Only
// the populations whose bit is set in `mask` (bit p: population p, flow
// 0..18, energy 19..25) are written.
template <class St, bool kOff32, typename Src>
__global__ __launch_bounds__(256) void k_unstream(char *__restrict__ dst,
                                                  Geometry<typename St::T> geo, Src srcS,
                                                  uint32_t mask)
{
    using T = typename St::T;
    using SF = typename St::F;
    using SG = typename St::G;
    using A = Access<kOff32>;
    using Lt = Lat<St, kOff32>;
    using I = typename A::I;
    const int n = geo.n;
    const long long cells = (long long)n * n * n;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells)
        return;
    const int x = int(c % n), y = int((c / n) % n), z = int(c / ((long long)n * n));
    for (int i = 0; i < 19; ++i) {
        if (!((mask >> i) & 1u))
            continue;
        const int tx = x + ex19(i), ty = y + ey19(i), tz = z + ez19(i);
        const bool in = tx >= 0 && tx < n && ty >= 0 && ty < n && tz >= 0 && tz < n;
        double v = in ? srcS.f(i, tx + n * (ty + n * tz)) : srcS.f(opp19(i), int(c));
        A::template st<SF>(dst, Lt::f(I(c), i), Codec<SF>::enc(T(v), T(inv_w19(i))));
    }
    const double th_lin = double(geo.theta_hot) +
                          double(geo.theta_cold - geo.theta_hot) * (y + 0.5) / n;
    const int gx[7] = {0, 1, -1, 0, 0, 0, 0}, gy[7] = {0, 0, 0, 1, -1, 0, 0},
              gz[7] = {0, 0, 0, 0, 0, 1, -1}, go[7] = {0, 2, 1, 4, 3, 6, 5};
    for (int i = 0; i < 7; ++i) {
        if (!((mask >> (19 + i)) & 1u))
            continue;
        const int tx = x + gx[i], ty = y + gy[i], tz = z + gz[i];
        double v;
        if (tx >= 0 && tx < n && ty >= 0 && ty < n && tz >= 0 && tz < n) {
            v = srcS.g(i, tx + n * (ty + n * tz));
        } else {
            const double s_in = srcS.g(go[i], int(c));
            bool dir;
            double tw = 0.0;
            if (ty < 0) { dir = true; tw = double(geo.theta_hot); }
            else if (ty >= n) { dir = true; tw = double(geo.theta_cold); }
            else if (tx < 0 || tx >= n) { dir = x_wall_dirichlet(geo.wall_type); tw = th_lin; }
            else { dir = z_wall_dirichlet(geo.wall_type); tw = th_lin; }
            // S_ibar = -P_i + 2 w theta_W (Dirichlet) or P_i (adiabatic)
            v = dir ? 2.0 * w7(go[i]) * tw - s_in : s_in;
        }
        const T inv_w = St::kScaledG ? T(inv_w7(i)) * geo.inv_escale : T(inv_w7(i));
        A::template st<SG>(dst, Lt::g(I(c), i), Codec<SG>::enc(T(v), inv_w));
    }
}

// ------------------------------------------------------------ read kernels
// Macroscopic fields at time t: rho, u = j / rho, theta (double outputs).
// Guo's forcing reports u_z = j_z / rho + vshift (theta - theta_ref) with
// vshift = g beta / 2 (the half-force velocity); vshift = 0 otherwise.
template <class St, bool kOff32>
__global__ __launch_bounds__(256) void k_macro(const char *__restrict__ src,
                                               Geometry<typename St::T> geo, double vshift,
                                               double theta_ref, double *rho, double *ux,
                                               double *uy, double *uz, double *theta)
{
    using T = typename St::T;
    const int n = geo.n;
    const long long cells = (long long)n * n * n;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells)
        return;
    const int x = int(c % n), y = int((c / n) % n), z = int(c / ((long long)n * n));
    T f[19], g[7];
    pull<St, kOff32>(src, geo, x, y, z, f, g);
    double dr = 0.0, j[3] = {0.0, 0.0, 0.0}, th = 0.0;
    for (int i = 0; i < 19; ++i) {
        dr += double(f[i]);
        j[0] += ex19(i) * double(f[i]);
        j[1] += ey19(i) * double(f[i]);
        j[2] += ez19(i) * double(f[i]);
    }
    for (int i = 0; i < 7; ++i)
        th += double(g[i]);
    const double r = 1.0 + dr;
    if (rho) rho[c] = r;
    if (ux) ux[c] = j[0] / r;
    if (uy) uy[c] = j[1] / r;
    if (uz) uz[c] = vshift != 0.0 ? j[2] / r + vshift * (th - theta_ref) : j[2] / r;
    if (theta) theta[c] = th;
}

// Populations first .. first + count - 1 (flow 0..18, energy 19..25) at
// time t as plain doubles: out[(p - first) * n^3 + c].
template <class St, bool kOff32>
__global__ __launch_bounds__(256) void k_pops(const char *__restrict__ src,
                                              Geometry<typename St::T> geo, int first, int count,
                                              double *out)
{
    using T = typename St::T;
    const int n = geo.n;
    const long long cells = (long long)n * n * n;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells)
        return;
    const int x = int(c % n), y = int((c / n) % n), z = int(c / ((long long)n * n));
    T f[19], g[7];
    pull<St, kOff32>(src, geo, x, y, z, f, g);
    for (int k = 0; k < count; ++k) {
        const int p = first + k;
        out[(size_t)k * cells + c] = p < 19 ? w19(p) + double(f[p]) : double(g[p - 19]);
    }
}

// --------------------------------------------------------- Nusselt number
// Wavefront-wide reductions (64 lanes on CDNA).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Combine 4 per-lane accumulators (sum, line, max, bad) across the block:
// wavefront shuffles, then the first lane of each wave through LDS.  The
// block-wide result is valid in thread 0.
__device__ __forceinline__ void block_reduce4(double &sum, double &line, double &mx, double &bad)
{
    __shared__ double red[4][16];
    sum = wave_sum(sum);
    line = wave_sum(line);
    mx = wave_max(mx);
    bad = wave_sum(bad);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = sum;
        red[1][wv] = line;
        red[2][wv] = mx;
        red[3][wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0, l = 0.0, m = -1.0e300, b = 0.0;
        for (int k = 0; k < nw; ++k) {
            s += red[0][k];
            l += red[1][k];
            m = fmax(m, red[2][k]);
            b += red[3][k];
        }
        sum = s;
        line = l;
        mx = m;
        bad = b;
    }
}

// One block per z row of the hot wall (y = 0).  Local Nu (Eq. 39) from the
// wall-adjacent nodes, by stencil (LBMX_NU_*):
//   0  second order, dtheta/dy = (9 th0 - th1 - 8 th_w)/3;
//   1  first order, dtheta/dy = 2 (th0 - th_w);
//   2  energy crossing the wall links, q = 2 (g_+y - th_w / 8), as -q / D_yy
//      (g_+y at the wall node is the population that came from the wall).
// partial[z] = {sum over x, X = 0.5 line contribution, max, non-finite count}.
template <class St, bool kOff32>
__global__ __launch_bounds__(256) void k_nu_rows(const char *__restrict__ src,
                                                 Geometry<typename St::T> geo, double theta_hot,
                                                 int stencil, double d_yy, double *partial,
                                                 double *map)
{
    using T = typename St::T;
    const int n = geo.n;
    const int z = blockIdx.x;
    double sum = 0.0, line = 0.0, mx = -1.0e300, bad = 0.0;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        T f[19], g0[7], g1[7];
        pull<St, kOff32>(src, geo, x, 0, z, f, g0);
        double th0 = 0.0, th1 = 0.0;
        for (int i = 0; i < 7; ++i)
            th0 += double(g0[i]);
        double nu;
        if (stencil == 1) {
            nu = -double(n) * 2.0 * (th0 - theta_hot);
        } else if (stencil == 2) {
            nu = double(n) * 2.0 * (double(g0[3]) - 0.125 * theta_hot) / d_yy;
        } else {
            pull<St, kOff32>(src, geo, x, 1, z, f, g1);
            for (int i = 0; i < 7; ++i)
                th1 += double(g1[i]);
            nu = -double(n) * (9.0 * th0 - th1 - 8.0 * theta_hot) / 3.0;
        }
        if (map)
            map[x + (size_t)n * z] = nu;
        if (!isfinite(nu)) {
            bad += 1.0;
            continue;
        }
        sum += nu;
        mx = fmax(mx, nu);
        if (n & 1) {
            if (x == n / 2) line += nu;
        } else if (x == n / 2 - 1 || x == n / 2) {
            line += 0.5 * nu;
        }
    }
    block_reduce4(sum, line, mx, bad);
    if (threadIdx.x == 0) {
        partial[4 * z + 0] = sum;
        partial[4 * z + 1] = line;
        partial[4 * z + 2] = mx;
        partial[4 * z + 3] = bad;
    }
}

// Combine the per-row partials in a fixed order: out = {Nu_3D, Nu_2D, Nu_max, bad}.
// (A template only so that every translation unit may include this header.)
template <int kUnused = 0>
__global__ __launch_bounds__(256) void k_nu_final(const double *partial, int n, double *out)
{
    double sum = 0.0, line = 0.0, mx = -1.0e300, bad = 0.0;
    for (int z = threadIdx.x; z < n; z += blockDim.x) {
        sum += partial[4 * z + 0];
        line += partial[4 * z + 1];
        mx = fmax(mx, partial[4 * z + 2]);
        bad += partial[4 * z + 3];
    }
    block_reduce4(sum, line, mx, bad);
    if (threadIdx.x == 0) {
        out[0] = sum / (double(n) * double(n));  // Eq. (40), midpoint rule
        out[1] = line / double(n);               // Eq. (41), midpoint rule
        out[2] = mx;
        out[3] = bad;
    }
}

}  // namespace lbmx
