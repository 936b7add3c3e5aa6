// host.hpp -- host-side helpers shared by the single-cavity and batch
// entry points of the C-ABI: parameter derivation and validation (Sec. 4,
// Eq. 38; Eqs. 26, 36), relaxation-rate tables, lattice layout, and the
// launchers of the initialisation / readback / Nusselt kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../include/lbmx.h"
#include "kernels.hpp"

namespace lbmx {
namespace host {

// Record a thread-local error message (lbmx_last_error) and return s.
lbmx_status fail(lbmx_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(LBMX_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Element bytes of the flow (D3Q19) and energy (D3Q7) populations.
inline size_t flow_size(int32_t s)
{
    switch (s) {
    case LBMX_F64: return 8;
    case LBMX_F32: return 4;
    case LBMX_F16:
    case LBMX_BF16:
    case LBMX_F16_F32:
    case LBMX_BF16_F32:
    case LBMX_F16_I16: return 2;
    default: return 0;
    }
}
inline size_t energy_size(int32_t s)
{
    switch (s) {
    case LBMX_F64: return 8;
    case LBMX_F32:
    case LBMX_F16_F32:
    case LBMX_BF16_F32: return 4;
    case LBMX_F16:
    case LBMX_BF16:
    case LBMX_F16_I16: return 2;
    default: return 0;
    }
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Derived {
    double u_c, gbeta, nu, alpha, s_nu, tau_t;
    double s[19], tau[7];
    double tbar[6];   // tau-bar block of Q^-1 (Eq. 35): xx, yy, zz, xy, xz, yz
    double d_yy;      // D_yy = epsilon (tau-bar_yy - 1/2), Eq. (36) solved for D
};

// Sec. 4, Eq. (38): Ma = u_c / c_s with c_s^2 = 1/3 (Eq. 13), u_c^2 = g beta dT H
// (dT = 1 in units of theta), Ra = g beta dT H^3 Pr / nu^2, Pr = nu / alpha.
// Eq. (26): s_nu = 1/(3 nu + 1/2).  Eq. (36): tau = 1/2 + alpha/epsilon, epsilon = 1/4.
inline lbmx_status derive(const lbmx_params *p, Derived *d)
{
    if (!p)
        return fail(LBMX_EINVAL, "params is NULL");
    if (p->n < 4 || p->n > 1024)
        return fail(LBMX_EINVAL, "n = %d outside [4, 1024]", p->n);
    if (p->wall_type < 1 || p->wall_type > 3)
        return fail(LBMX_EINVAL, "wall_type = %d not in {1, 2, 3}", p->wall_type);
    if (!(p->ra > 0) || !std::isfinite(p->ra))
        return fail(LBMX_EINVAL, "Ra must be positive and finite");
    if (!(p->pr > 0) || !std::isfinite(p->pr))
        return fail(LBMX_EINVAL, "Pr must be positive and finite");
    if (!(p->ma > 0) || !(p->ma <= 0.5))
        return fail(LBMX_EINVAL, "Ma = %g outside (0, 0.5]", p->ma);
    if (!std::isfinite(p->theta_hot) || !std::isfinite(p->theta_cold) ||
        !std::isfinite(p->theta_ref) || !std::isfinite(p->buoyancy_scale))
        return fail(LBMX_EINVAL, "non-finite temperature or buoyancy parameter");
    if (flow_size(p->storage) == 0)
        return fail(LBMX_EINVAL, "storage = %d not a lbmx_storage", p->storage);
    const double u_c = p->ma * std::sqrt(1.0 / 3.0);
    d->u_c = u_c;
    d->gbeta = u_c * u_c / p->n;
    d->nu = u_c * p->n * std::sqrt(p->pr / p->ra);
    d->alpha = d->nu / p->pr;
    d->s_nu = 1.0 / (3.0 * d->nu + 0.5);
    d->tau_t = 0.5 + 4.0 * d->alpha;
    if (p->custom_rates) {
        for (int k = 0; k < 19; ++k) {
            if (!(p->s[k] >= 0.0 && p->s[k] <= 2.0))
                return fail(LBMX_EINVAL, "custom s[%d] = %g outside [0, 2]", k, p->s[k]);
            d->s[k] = p->s[k];
        }
        for (int k = 0; k < 7; ++k) {
            if (!(p->tau[k] > 0.0) || !std::isfinite(p->tau[k]))
                return fail(LBMX_EINVAL, "custom tau[%d] = %g not positive", k, p->tau[k]);
            d->tau[k] = p->tau[k];
        }
        if (!(d->tau[1] > 0.5 && d->tau[2] > 0.5 && d->tau[3] > 0.5))
            return fail(LBMX_EINVAL, "custom diffusion rates need tau > 1/2");
    } else {
        if (!(d->s_nu > 0.0 && d->s_nu < 2.0))
            return fail(LBMX_EINVAL, "s_nu = %g outside (0, 2)", d->s_nu);
        if (!(d->tau_t > 0.5))
            return fail(LBMX_EINVAL, "tau_T = %g not above 1/2", d->tau_t);
        const double sn = d->s_nu;
        const double s[19] = {1.0, 1.19, 1.4, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, sn,
                              1.4, sn,   1.4, sn,  sn,  sn,  1.98, 1.98, 1.98};
        for (int k = 0; k < 19; ++k)
            d->s[k] = s[k];
        const double tau[7] = {1.0, d->tau_t, d->tau_t, d->tau_t, 1.0, 1.0, 1.0};
        for (int k = 0; k < 7; ++k)
            d->tau[k] = tau[k];
    }
    if (p->force_model < LBMX_FORCE_EQ15 || p->force_model > LBMX_FORCE_GUO)
        return fail(LBMX_EINVAL, "force_model = %d not a LBMX_FORCE_* value", p->force_model);
    if (p->nu_stencil < LBMX_NU_SECOND_ORDER || p->nu_stencil > LBMX_NU_WALL_FLUX)
        return fail(LBMX_EINVAL, "nu_stencil = %d not a LBMX_NU_* value", p->nu_stencil);
    // tau-bar block: the diagonal tau_1..tau_3, or Eq. (36) with D = alpha A.
    const double *A = p->aniso;
    bool aniso = false;
    for (int k = 0; k < 6; ++k) {
        if (!std::isfinite(A[k]))
            return fail(LBMX_EINVAL, "aniso[%d] is not finite", k);
        aniso = aniso || A[k] != 0.0;
    }
    if (aniso) {
        if (p->custom_rates)
            return fail(LBMX_EINVAL, "aniso and custom_rates cannot be combined");
        // positive definite: leading principal minors > 0 (xx, yy, zz, xy, xz, yz)
        const double m1 = A[0], m2 = A[0] * A[1] - A[3] * A[3];
        const double m3 = A[0] * (A[1] * A[2] - A[5] * A[5]) - A[3] * (A[3] * A[2] - A[5] * A[4]) +
                          A[4] * (A[3] * A[5] - A[1] * A[4]);
        if (!(m1 > 0.0 && m2 > 0.0 && m3 > 0.0))
            return fail(LBMX_EINVAL, "aniso tensor is not positive definite");
        for (int k = 0; k < 6; ++k)
            d->tbar[k] = (k < 3 ? 0.5 : 0.0) + d->alpha * A[k] / 0.25;
    } else {
        d->tbar[0] = d->tau[1];
        d->tbar[1] = d->tau[2];
        d->tbar[2] = d->tau[3];
        d->tbar[3] = d->tbar[4] = d->tbar[5] = 0.0;
    }
    d->d_yy = 0.25 * (d->tbar[1] - 0.5);
    return LBMX_OK;
}

template <typename T>
Rates<T> make_rates(const lbmx_params *p, const Derived &d)
{
    // s_k / |M_k|^2 with the squared row norms of Eq. (21) (rows orthogonal).
    Rates<T> r;
    r.e = T(d.s[1] / 2394.0);
    r.eps = T(d.s[2] / 252.0);
    r.qx = T(d.s[4] / 40.0);
    r.qy = T(d.s[6] / 40.0);
    r.qz = T(d.s[8] / 40.0);
    r.pxx = T(d.s[9] / 36.0);
    r.pixx = T(d.s[10] / 72.0);
    r.pww = T(d.s[11] / 12.0);
    r.piww = T(d.s[12] / 24.0);
    r.pxy = T(d.s[13] / 4.0);
    r.pyz = T(d.s[14] / 4.0);
    r.pxz = T(d.s[15] / 4.0);
    r.mx = T(d.s[16] / 8.0);
    r.my = T(d.s[17] / 8.0);
    r.mz = T(d.s[18] / 8.0);
    // Guo's forcing: (1 - s_k/2) / |M_k|^2, same rows.
    const int rows[15] = {1, 2, 4, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18};
    const double norms[15] = {2394, 252, 40, 40, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};
    T *h[15] = {&r.he, &r.heps, &r.hqx, &r.hqy, &r.hqz, &r.hpxx, &r.hpixx, &r.hpww,
                &r.hpiww, &r.hpxy, &r.hpyz, &r.hpxz, &r.hmx, &r.hmy, &r.hmz};
    for (int k = 0; k < 15; ++k)
        *h[k] = T((1.0 - 0.5 * d.s[rows[k]]) / norms[k]);
    // Q = (Q^-1)^-1 (Eq. 35) over |N_k|^2 of Eq. (32) (2 for n_1..n_3).  The
    // tau-bar block is inverted as a symmetric 3x3 (cofactors); a diagonal
    // block takes plain reciprocals.
    const double *b = d.tbar;  // xx, yy, zz, xy, xz, yz
    if (b[3] == 0.0 && b[4] == 0.0 && b[5] == 0.0) {
        r.q11 = T(1.0 / b[0] / 2.0);
        r.q22 = T(1.0 / b[1] / 2.0);
        r.q33 = T(1.0 / b[2] / 2.0);
        r.q12 = r.q13 = r.q23 = T(0);
    } else {
        const double c11 = b[1] * b[2] - b[5] * b[5], c22 = b[0] * b[2] - b[4] * b[4];
        const double c33 = b[0] * b[1] - b[3] * b[3];
        const double c12 = b[4] * b[5] - b[3] * b[2], c13 = b[3] * b[5] - b[4] * b[1];
        const double c23 = b[3] * b[4] - b[0] * b[5];
        const double det = b[0] * c11 + b[3] * c12 + b[4] * c13;
        r.q11 = T(c11 / det / 2.0);
        r.q22 = T(c22 / det / 2.0);
        r.q33 = T(c33 / det / 2.0);
        r.q12 = T(c12 / det / 2.0);
        r.q13 = T(c13 / det / 2.0);
        r.q23 = T(c23 / det / 2.0);
    }
    r.t4 = T(1.0 / d.tau[4] / 42.0);
    r.t5 = T(1.0 / d.tau[5] / 12.0);
    r.t6 = T(1.0 / d.tau[6] / 4.0);
    r.gbeta = T(d.gbeta * p->buoyancy_scale);
    r.theta_ref = T(p->theta_ref);
    return r;
}

struct Layout {
    size_t slab_nodes;   // nodes per slab, 2^slab_shift_for(flow element bytes)
    size_t lattice;      // bytes per lattice
    size_t scratch_off;  // byte offset of the Nu scratch
    size_t total;
};

inline Layout layout_of(const lbmx_params *p)
{
    Layout L;
    const size_t cells = (size_t)p->n * p->n * p->n;
    L.slab_nodes = size_t(1) << slab_shift_for(flow_size(p->storage));
    const size_t slabs = (cells + L.slab_nodes - 1) / L.slab_nodes;
    L.lattice = slabs * L.slab_nodes * (19 * flow_size(p->storage) + 7 * energy_size(p->storage));
    L.scratch_off = 2 * L.lattice;
    L.total = L.scratch_off + align_up(sizeof(double) * (4 * (size_t)p->n + 8), 256);
    return L;
}


// A lattice seen by the launchers: `lat` is the lattice holding the current
// state, `off32` selects 32-bit offsets.  `spare` is the cavity's other
// lattice (spare_bytes long): the next step overwrites all of it, so between
// steps it serves as the staging buffer of transfers and readbacks, which
// therefore allocate no device memory.  A lattice holds at least 52 bytes
// per node (26 16-bit populations), i.e. 6 doubles per node.
struct View {
    char *lat;
    char *spare;
    size_t spare_bytes;
    int n, wall_type;
    double theta_hot, theta_cold;
    bool off32;
    hipStream_t stream;
    double vshift;     // g beta / 2 for Guo's forcing (reported velocity), else 0
    double theta_ref;
    int nu_stencil;
    double d_yy;       // for the wall-flux Nu stencil
};

inline View make_view(char *lat, char *spare, size_t spare_bytes, const lbmx_params &p,
                      const Derived &d, bool off32, hipStream_t stream)
{
    View v;
    v.lat = lat;
    v.spare = spare;
    v.spare_bytes = spare_bytes;
    v.n = p.n;
    v.wall_type = p.wall_type;
    v.theta_hot = p.theta_hot;
    v.theta_cold = p.theta_cold;
    v.off32 = off32;
    v.stream = stream;
    v.vshift = p.force_model == LBMX_FORCE_GUO ? 0.5 * d.gbeta * p.buoyancy_scale : 0.0;
    v.theta_ref = p.theta_ref;
    v.nu_stencil = p.nu_stencil;
    v.d_yy = d.d_yy;
    return v;
}

// Theta of the fixed-point energy code: the power of two at or above
// 2 max(|theta_hot|, |theta_cold|) (1 when both are 0).
inline double energy_scale(double theta_hot, double theta_cold)
{
    const double m = 2.0 * std::max(std::fabs(theta_hot), std::fabs(theta_cold));
    return m > 0.0 ? std::exp2(std::ceil(std::log2(m))) : 1.0;
}

template <class St>
Geometry<typename St::T> geometry(const View &v)
{
    using T = typename St::T;
    Geometry<T> g;
    g.n = v.n;
    g.wall_type = v.wall_type;
    g.theta_hot = T(v.theta_hot);
    g.theta_cold = T(v.theta_cold);
    g.step = 0;
    const double es = St::kScaledG ? energy_scale(v.theta_hot, v.theta_cold) : 1.0;
    g.escale = T(es);
    g.inv_escale = T(1.0 / es);
    return g;
}

constexpr uint32_t kAllPops = (1u << 26) - 1;

template <class St, typename Src>
lbmx_status launch_unstream(const View &v, const Src &src, uint32_t mask = kAllPops)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    if (v.off32)
        hipLaunchKernelGGL((k_unstream<St, true, Src>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), src, mask);
    else
        hipLaunchKernelGGL((k_unstream<St, false, Src>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), src, mask);
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

template <class St>
lbmx_status launch_macro(const View &v, double *r, double *u, double *w3, double *w, double *th)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    if (v.off32)
        hipLaunchKernelGGL((k_macro<St, true>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), v.vshift, v.theta_ref, r, u, w3, w, th);
    else
        hipLaunchKernelGGL((k_macro<St, false>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), v.vshift, v.theta_ref, r, u, w3, w, th);
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

template <class St>
lbmx_status launch_pops(const View &v, int first, int count, double *out)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    if (v.off32)
        hipLaunchKernelGGL((k_pops<St, true>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), first, count, out);
    else
        hipLaunchKernelGGL((k_pops<St, false>), dim3(blocks), dim3(256), 0, v.stream, v.lat,
                           geometry<St>(v), first, count, out);
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

// Doubles per node the spare lattice can stage (at least 6).
inline size_t spare_doubles(const View &v)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    return v.spare_bytes / (sizeof(double) * cells);
}

// Host population array of population p (flow 0..18, energy 19..25).
template <typename D>
D *host_pop(D *f, D *g, int p, size_t cells)
{
    return p < 19 ? f + (size_t)p * cells : g + (size_t)(p - 19) * cells;
}

// Populations of the current state to host (f: 19 n^3, g: 7 n^3 doubles;
// either may be null), in passes of as many populations as the spare
// lattice holds.  Synchronises the stream.
template <class St>
lbmx_status pops_to_host(const View &v, double *f, double *g)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    const int cap = int(std::min<size_t>(26, spare_doubles(v)));
    double *stage = reinterpret_cast<double *>(v.spare);
    const int lo = f ? 0 : 19, hi = g ? 26 : 19;
    for (int p0 = lo; p0 < hi; p0 += cap) {
        const int count = std::min(cap, hi - p0);
        lbmx_status s = launch_pops<St>(v, p0, count, stage);
        if (s != LBMX_OK)
            return s;
        for (int k = 0; k < count; ++k)
            HIP_TRY(hipMemcpyAsync(host_pop(f, g, p0 + k, cells), stage + (size_t)k * cells,
                                   cells * sizeof(double), hipMemcpyDeviceToHost, v.stream));
    }
    HIP_TRY(hipStreamSynchronize(v.stream));
    return LBMX_OK;
}

// State from host populations (f: 19 n^3, g: 7 n^3 doubles): each pass
// stages whole opposite pairs (i, ibar) in the spare lattice and unstreams
// those populations.  Synchronises the stream.
template <class St>
lbmx_status pops_from_host(const View &v, const double *f, const double *g)
{
    static const int pairs[14][2] = {{0, -1},  {1, 2},   {3, 4},   {5, 6},   {7, 10},
                                     {8, 9},   {11, 14}, {12, 13}, {15, 18}, {16, 17},
                                     {19, -1}, {20, 21}, {22, 23}, {24, 25}};
    const size_t cells = (size_t)v.n * v.n * v.n;
    const int cap = int(std::min<size_t>(26, spare_doubles(v)));
    double *stage = reinterpret_cast<double *>(v.spare);
    int q = 0;
    while (q < 14) {
        SourcePops src;
        src.buf = stage;
        src.cells = cells;
        for (int p = 0; p < 26; ++p)
            src.slot[p] = -1;
        uint32_t mask = 0;
        int used = 0;
        for (; q < 14; ++q) {
            const int need = pairs[q][1] < 0 ? 1 : 2;
            if (used + need > cap)
                break;
            for (int m = 0; m < need; ++m) {
                const int p = pairs[q][m];
                src.slot[p] = (signed char)used;
                mask |= 1u << p;
                HIP_TRY(hipMemcpyAsync(stage + (size_t)used * cells, host_pop(f, g, p, cells),
                                       cells * sizeof(double), hipMemcpyHostToDevice, v.stream));
                ++used;
            }
        }
        lbmx_status s = launch_unstream<St>(v, src, mask);
        if (s != LBMX_OK)
            return s;
    }
    HIP_TRY(hipStreamSynchronize(v.stream));
    return LBMX_OK;
}

// Macroscopic fields of the current state to host arrays (any may be null),
// staged in the spare lattice (5 doubles per node).  Synchronises the stream.
template <class St>
lbmx_status macro_to_host(const View &v, double *r, double *u, double *w3, double *w, double *th)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    double *host[5] = {r, u, w3, w, th};
    double *dev[5];
    for (int k = 0; k < 5; ++k)
        dev[k] = host[k] ? reinterpret_cast<double *>(v.spare) + k * cells : nullptr;
    lbmx_status s = launch_macro<St>(v, dev[0], dev[1], dev[2], dev[3], dev[4]);
    if (s != LBMX_OK)
        return s;
    for (int k = 0; k < 5; ++k)
        if (host[k])
            HIP_TRY(hipMemcpyAsync(host[k], dev[k], cells * sizeof(double), hipMemcpyDeviceToHost,
                                   v.stream));
    HIP_TRY(hipStreamSynchronize(v.stream));
    return LBMX_OK;
}

// Nusselt reduction; `scratch` holds 4 n + 4 doubles, the result {Nu_3D,
// Nu_2D, Nu_max, non-finite count} lands at scratch + 4 n.
template <class St>
lbmx_status launch_nu(const View &v, double *scratch, double *map)
{
    const int n = v.n;
    double *out = scratch + 4 * (size_t)n;
    const int threads = n <= 64 ? 64 : (n <= 128 ? 128 : 256);
    if (v.off32)
        hipLaunchKernelGGL((k_nu_rows<St, true>), dim3(n), dim3(threads), 0, v.stream, v.lat,
                           geometry<St>(v), v.theta_hot, v.nu_stencil, v.d_yy, scratch, map);
    else
        hipLaunchKernelGGL((k_nu_rows<St, false>), dim3(n), dim3(threads), 0, v.stream, v.lat,
                           geometry<St>(v), v.theta_hot, v.nu_stencil, v.d_yy, scratch, map);
    hipLaunchKernelGGL(k_nu_final<0>, dim3(1), dim3(256), 0, v.stream, scratch, n, out);
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

template <class St>
lbmx_status unstream_rest(const View &v, const double *theta0)
{
    return launch_unstream<St>(v, SourceRest{theta0});
}

// Rest state with theta0 from the host (n^3 doubles, staged in the spare
// lattice; null = theta 0).  Synchronises the stream.
template <class St>
lbmx_status rest_from_host(const View &v, const double *theta0_host)
{
    const size_t cells = (size_t)v.n * v.n * v.n;
    const double *th = nullptr;
    if (theta0_host) {
        HIP_TRY(hipMemcpyAsync(v.spare, theta0_host, cells * sizeof(double), hipMemcpyHostToDevice,
                               v.stream));
        th = reinterpret_cast<const double *>(v.spare);
    }
    lbmx_status s = unstream_rest<St>(v, th);
    if (s != LBMX_OK)
        return s;
    HIP_TRY(hipStreamSynchronize(v.stream));
    return LBMX_OK;
}

template <class St, class E>
lbmx_status unstream_fields(const View &v, const E *u, const E *w2, const E *w, const E *th,
                            int src_n, double vscale, const E *rho)
{
    return launch_unstream<St>(v, SourceFields<E>{u, w2, w, th, src_n, v.n, E(vscale), rho});
}

// Device buffer released at scope exit (after the work using it completed:
// hipFree waits for the device).
struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
};

// Call fn<Store<SF, SG>>(args...) for a storage code.
#define LBMX_DISPATCH(storage, fn, ...)                                                        \
    ([&]() -> lbmx_status {                                                                    \
        switch (storage) {                                                                     \
        case LBMX_F64: return fn<Store<double, double>>(__VA_ARGS__);                          \
        case LBMX_F32: return fn<Store<float, float>>(__VA_ARGS__);                            \
        case LBMX_F16: return fn<Store<__half, __half>>(__VA_ARGS__);                          \
        case LBMX_BF16: return fn<Store<__hip_bfloat16, __hip_bfloat16>>(__VA_ARGS__);         \
        case LBMX_F16_F32: return fn<Store<__half, float>>(__VA_ARGS__);                       \
        case LBMX_BF16_F32: return fn<Store<__hip_bfloat16, float>>(__VA_ARGS__);              \
        case LBMX_F16_I16: return fn<Store<__half, Fix16>>(__VA_ARGS__);                       \
        default: return ::lbmx::host::fail(LBMX_EINVAL, "bad storage %d", int(storage));       \
        }                                                                                      \
    }())

// EINVAL unless both device buffers live on the current device.
inline lbmx_status check_same_device(const void *a, const void *b, const char *what)
{
    hipPointerAttribute_t pa, pb;
    HIP_TRY(hipPointerGetAttributes(&pa, a));
    HIP_TRY(hipPointerGetAttributes(&pb, b));
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (pa.device != pb.device || pb.device != dev)
        return fail(LBMX_EINVAL, "%s on devices %d and %d, current device %d", what, pa.device,
                    pb.device, dev);
    return LBMX_OK;
}

// dst's state at t = 0 from src's current state: src's rho, u = j / rho,
// theta (Eqs. 20, 25, 30) formed in FP64 on the device, resampled
// trilinearly onto dst's nodes (SourceFields<double>), velocities scaled by
// vscale and rho - 1 by vscale^2; f = f^eq(rho, u), g = g^eq(theta, u).
// Synchronises both streams; the 5 src.n^3 doubles of fields are staged in
// src's spare lattice (src's state is only read).
inline lbmx_status init_from_state(const View &dst, int32_t dst_storage, const View &src,
                                   int32_t src_storage, double vscale)
{
    const size_t mc = (size_t)src.n * src.n * src.n;
    double *f5 = reinterpret_cast<double *>(src.spare);
    lbmx_status s = LBMX_DISPATCH(src_storage, launch_macro, src, f5 + 4 * mc, f5, f5 + mc,
                                  f5 + 2 * mc, f5 + 3 * mc);
    if (s != LBMX_OK)
        return s;
    HIP_TRY(hipStreamSynchronize(src.stream));
    s = LBMX_DISPATCH(dst_storage, unstream_fields, dst, (const double *)f5,
                      (const double *)(f5 + mc), (const double *)(f5 + 2 * mc),
                      (const double *)(f5 + 3 * mc), src.n, vscale,
                      (const double *)(f5 + 4 * mc));
    if (s != LBMX_OK)
        return s;
    HIP_TRY(hipStreamSynchronize(dst.stream));
    return LBMX_OK;
}

template <class St>
lbmx_status unstream_two_fields(const View &v, const SourceTwoFields &src)
{
    return launch_unstream<St>(v, src);
}

// dst's state at t = 0 from wa (fields of a) + wb (fields of b): each
// source's rho, u = j / rho and theta formed in FP64 on the device (staged in
// its own spare lattice), sampled trilinearly onto dst's nodes with
// velocities scaled by sa / sb and rho - 1 by sa^2 / sb^2, combined;
// f = f^eq(rho, u), g = g^eq(theta, u).
// Synchronises the three streams; a and b are only read and must differ.
inline lbmx_status init_from_two_states(const View &dst, int32_t dst_storage, const View &a,
                                        int32_t a_storage, double wa, double sa, const View &b,
                                        int32_t b_storage, double wb, double sb)
{
    const View *src[2] = {&a, &b};
    const int32_t sto[2] = {a_storage, b_storage};
    SourceFields<double> sf[2];
    for (int k = 0; k < 2; ++k) {
        const View &v = *src[k];
        const size_t mc = (size_t)v.n * v.n * v.n;
        double *f5 = reinterpret_cast<double *>(v.spare);
        lbmx_status s = LBMX_DISPATCH(sto[k], launch_macro, v, f5 + 4 * mc, f5, f5 + mc,
                                      f5 + 2 * mc, f5 + 3 * mc);
        if (s != LBMX_OK)
            return s;
        sf[k] = SourceFields<double>{f5, f5 + mc, f5 + 2 * mc, f5 + 3 * mc, v.n, dst.n,
                                     k == 0 ? sa : sb, f5 + 4 * mc};
    }
    HIP_TRY(hipStreamSynchronize(a.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    lbmx_status s = LBMX_DISPATCH(dst_storage, unstream_two_fields, dst,
                                  SourceTwoFields{sf[0], sf[1], wa, wb});
    if (s != LBMX_OK)
        return s;
    HIP_TRY(hipStreamSynchronize(dst.stream));
    return LBMX_OK;
}

}  // namespace host
}  // namespace lbmx
