// batch.hpp -- one launch advancing many cavities of different size and
// parameters by one time step (same node update as k_step: pull streaming
// with the wall rules of Eqs. 6-10, double-MRT collision of Sec. 3).
//
// Work list: every active cavity's n^3 nodes are cut, in storage order, into
// tiles of blockDim.x consecutive nodes; tile t is {cavity, first node}.  A
// block takes tiles blockIdx.x, blockIdx.x + gridDim.x, ... (grid-stride
// "persistent" blocks when gridDim.x is smaller than the tile count, one
// tile per block when equal).  Consecutive nodes of a tile are consecutive
// in every population segment (up to a slab boundary), so loads and stores
// stay coalesced across row boundaries, and every wavefront is full except
// at the end of a cavity.  The per-cavity table (lattice pointers, geometry,
// relaxation rates) is read with wavefront-uniform loads.
#pragma once

#include "kernels.hpp"

namespace lbmx {

template <typename T>
struct BatchCav {
    char *lat[2];        // the cavity's two lattices
    Geometry<T> geo;
    Rates<T> rates;
    uint32_t cells;      // n^3 (< 2^24)
    float inv_n;         // 1/n, for the quotient below
};

struct Tile {
    uint32_t cav;        // index into the cavity table
    uint32_t start;      // first node (flat index x + n (y + n z))
};

// floor(c / n) for c < 2^24: the float quotient is within 1/2 of the true
// one, so a single correction by one is exact.
__device__ __forceinline__ uint32_t div_small(uint32_t c, uint32_t n, float inv_n)
{
    uint32_t q = uint32_t(float(c) * inv_n);
    const int32_t r = int32_t(c) - int32_t(q * n);
    if (r < 0)
        q -= 1;
    else if (r >= int32_t(n))
        q += 1;
    return q;
}

// Each cavity's time step lives on the device, in two arrays used by turns:
// a launch of parity p reads cavity k's step from t_in[k] (the stochastic-
// rounding key of the fixed-point energy format, the same key a lone
// cavity uses at that step) and the block that owns the cavity's first
// tile writes step + 1 to t_out[k], which the next launch (parity 1 - p)
// reads.  No launch writes what it reads, so a captured graph replays with
// advancing steps.
template <class St, int kForce>
__global__ __launch_bounds__(1024) void k_step_batch(const BatchCav<typename St::T> *__restrict__ cavs,
                                                     const Tile *__restrict__ tiles, uint32_t ntiles,
                                                     int parity, const uint32_t *__restrict__ t_in,
                                                     uint32_t *__restrict__ t_out)
{
    using T = typename St::T;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tile = tiles[t];
        const BatchCav<T> *cv = cavs + tile.cav;
        const uint32_t step = t_in[tile.cav];
        if (tile.start == 0 && threadIdx.x == 0)
            t_out[tile.cav] = step + 1u;
        const uint32_t c = tile.start + threadIdx.x;
        if (c >= cv->cells)
            continue;
        const uint32_t n = uint32_t(cv->geo.n);
        const uint32_t q = div_small(c, n, cv->inv_n);
        const uint32_t z = div_small(q, n, cv->inv_n);
        const int x = int(c - q * n), y = int(q - z * n);
        const Geometry<T> geo = cv->geo;
        T f[19], g[7];
        pull<St, true>(cv->lat[parity], geo, x, y, int(z), f, g);
        collide<T, kForce>(f, g, cv->rates);
        put<St, true>(cv->lat[parity ^ 1], c, step, f, g, geo.inv_escale);
    }
}

// Trilinear resampling of node-centred fields (n^3, x fastest) onto an
// m^3 node-centred grid covering the same cube; positions outside the
// outermost node centres are clamped to them.  out[k][m^3] for the fields
// in[k][n^3], k < nf.
__global__ __launch_bounds__(256) void k_resample(const double *__restrict__ in, int n, int nf,
                                                  float *__restrict__ out, int m)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long mc = (long long)m * m * m;
    if (c >= mc)
        return;
    const int o[3] = {int(c % m), int((c / m) % m), int(c / ((long long)m * m))};
    int i0[3], i1[3];
    double fr[3];
    for (int d = 0; d < 3; ++d) {
        double p = (o[d] + 0.5) * double(n) / double(m) - 0.5;
        p = fmin(fmax(p, 0.0), double(n - 1));
        int k = int(floor(p));
        if (k > n - 2) k = n - 2 < 0 ? 0 : n - 2;
        i0[d] = k;
        i1[d] = k + 1 < n ? k + 1 : n - 1;
        fr[d] = p - k;
    }
    const size_t cells = (size_t)n * n * n;
    for (int k = 0; k < nf; ++k) {
        const double *a = in + (size_t)k * cells;
        auto at = [&](int x, int y, int z) { return a[x + (size_t)n * (y + (size_t)n * z)]; };
        const double c00 = at(i0[0], i0[1], i0[2]) * (1 - fr[0]) + at(i1[0], i0[1], i0[2]) * fr[0];
        const double c10 = at(i0[0], i1[1], i0[2]) * (1 - fr[0]) + at(i1[0], i1[1], i0[2]) * fr[0];
        const double c01 = at(i0[0], i0[1], i1[2]) * (1 - fr[0]) + at(i1[0], i0[1], i1[2]) * fr[0];
        const double c11 = at(i0[0], i1[1], i1[2]) * (1 - fr[0]) + at(i1[0], i1[1], i1[2]) * fr[0];
        const double c0 = c00 * (1 - fr[1]) + c10 * fr[1];
        const double c1 = c01 * (1 - fr[1]) + c11 * fr[1];
        out[(size_t)k * mc + c] = float(c0 * (1 - fr[2]) + c1 * fr[2]);
    }
}

}  // namespace lbmx
