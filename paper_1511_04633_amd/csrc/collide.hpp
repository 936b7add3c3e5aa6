// collide.hpp -- per-node double-MRT collision for the MI355X step kernel.
//
// Li, Yang & Zhang (arXiv:1511.04633), Sec. 3.  D3Q19 flow lattice with the
// moment basis of Eqs. (21)-(22), equilibrium moments of Eq. (24) (rho_0 = 1),
// diagonal relaxation S (Eqs. 23, 26), Boussinesq force of Eqs. (15)-(17)
// added after the collision (Eq. 14) or, as an alternative, Guo's forcing;
// D3Q7 energy lattice with N of Eq. (32), n^eq of Eq. (33) and Q of
// Eqs. (35)-(36), whose first-moment block may be a full symmetric 3x3
// (anisotropic diffusion).
//
// The transform is never formed as a matrix.  Its rows are orthogonal
// integer polynomials of the velocities, so m = M f is evaluated as sums and
// differences of opposite-direction pairs, and M^-1 = M^T diag(1/|M_k|^2)
// applies the same pair structure backwards.  The rows of the conserved
// moments (rho, j) relax an exact zero and are skipped.  p_xy is the moment
// e_x e_y named by Eq. (22); the matrix printed as Eq. (21) has a wrong sign
// pattern in that row (it would make M singular).
//
// Populations enter as offsets from rest equilibrium: df_i = f_i - w_i.
// Since M w = m^eq(rho = 1, j = 0) = (1, -11, 3, 0, ...), the moment
// deviations m - m^eq are formed from small numbers only, which keeps FP32
// arithmetic accurate (the signal u ~ 1e-2 would otherwise sit three digits
// below the O(w_i) populations).
//
// Direction order (0-based, paper's Eq. 12):
//   0 rest; 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z;
//   7 (+1,+1,0)  8 (-1,+1,0)  9 (+1,-1,0) 10 (-1,-1,0)
//  11 (+1,0,+1) 12 (-1,0,+1) 13 (+1,0,-1) 14 (-1,0,-1)
//  15 (0,+1,+1) 16 (0,-1,+1) 17 (0,+1,-1) 18 (0,-1,-1)
// D3Q7 (Eq. 28): 0 rest; 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z.
#pragma once

#include <hip/hip_runtime.h>

namespace lbmx {

// Relaxation rate of each non-conserved moment divided by the squared norm
// of its row of M (the diagonal of M M^T), and likewise for the D3Q7 moments.
template <typename T>
struct Rates {
    T e, eps, qx, qy, qz, pxx, pixx, pww, piww, pxy, pyz, pxz, mx, my, mz;
    // (1 - s_k/2) / |M_k|^2 in the same order: Guo's forcing (force model 2)
    T he, heps, hqx, hqy, hqz, hpxx, hpixx, hpww, hpiww, hpxy, hpyz, hpxz, hmx, hmy, hmz;
    // Q = (Q^-1)^-1 (Eq. 35) over |N_k|^2: the symmetric 3x3 block of the
    // first moments n_1..n_3 (anisotropic diffusion, Eq. 36) and n_4..n_6
    T q11, q22, q33, q12, q13, q23;
    T t4, t5, t6;
    T gbeta;                    // g beta per unit theta (buoyancy scale applied)
    T theta_ref;
};

// Force models: how the buoyancy G = g beta (theta - theta_ref) e_z enters.
//   0  Eq. (15) with the density in f^eq: F_i = 3 G (e_iz - u_z) f^eq_i(rho, u)
//   1  the same divided by rho (force density G instead of rho G)
//   2  Guo's forcing in moment space: u = (j + rho G / 2) / rho in the
//      equilibria, and (I - S/2) M Fbar added to the relaxation, with
//      Fbar_i = w_i rho [3 (e_i - u) + 9 (e_i . u) e_i] . G.

// Equilibrium of Eq. (17) without the rho w_i factor: 1 + 3 t + 4.5 t^2 - 1.5 u.u,
// with c0 = 1 - 1.5 u.u and t = e_i . u.
template <typename T>
__device__ __forceinline__ T feq_poly(T c0, T t)
{
    return c0 + t * (T(3) + T(4.5) * t);
}

// m = M x for a 19-vector x (Eqs. 21-22), from pair sums and differences.
// rho and j are the conserved rows; the other 15 in the order of Rates.
template <typename T>
struct Moments {
    T rho, jx, jy, jz;
    T e, eps, qx, qy, qz, pxx, pixx, pww, piww, pxy, pxz, pyz, mx, my, mz;
};

template <typename T>
__device__ __forceinline__ Moments<T> moments(const T x[19])
{
    const T Sx = x[1] + x[2], Dx = x[1] - x[2];
    const T Sy = x[3] + x[4], Dy = x[3] - x[4];
    const T Sz = x[5] + x[6], Dz = x[5] - x[6];
    // xy plane: 7 (+,+) <-> 10 (-,-), 8 (-,+) <-> 9 (+,-)
    const T a1 = x[7] + x[10], b1 = x[7] - x[10], c1 = x[8] + x[9], d1 = x[8] - x[9];
    // xz plane: 11 (+,+) <-> 14 (-,-), 12 (-,+) <-> 13 (+,-)
    const T a2 = x[11] + x[14], b2 = x[11] - x[14], c2 = x[12] + x[13], d2 = x[12] - x[13];
    // yz plane: 15 (+,+) <-> 18 (-,-), 16 (-,+) <-> 17 (+,-)
    const T a3 = x[15] + x[18], b3 = x[15] - x[18], c3 = x[16] + x[17], d3 = x[16] - x[17];

    const T sxy = a1 + c1, sxz = a2 + c2, syz = a3 + c3;
    const T jx_xy = b1 - d1, jy_xy = b1 + d1;
    const T jx_xz = b2 - d2, jz_xz = b2 + d2;
    const T jy_yz = b3 - d3, jz_yz = b3 + d3;

    const T s_ax = Sx + Sy + Sz;
    const T s_dg = sxy + sxz + syz;

    Moments<T> m;
    m.rho = x[0] + s_ax + s_dg;
    m.jx = Dx + jx_xy + jx_xz;
    m.jy = Dy + jy_xy + jy_yz;
    m.jz = Dz + jz_xz + jz_yz;
    m.e = T(-30) * x[0] - T(11) * s_ax + T(8) * s_dg;
    m.eps = T(12) * x[0] - T(4) * s_ax + s_dg;
    m.qx = T(-4) * Dx + jx_xy + jx_xz;
    m.qy = T(-4) * Dy + jy_xy + jy_yz;
    m.qz = T(-4) * Dz + jz_xz + jz_yz;
    m.pxx = T(2) * Sx - Sy - Sz + sxy + sxz - T(2) * syz;
    m.pixx = T(-4) * Sx + T(2) * (Sy + Sz) + sxy + sxz - T(2) * syz;
    m.pww = Sy - Sz + sxy - sxz;
    m.piww = T(2) * (Sz - Sy) + sxy - sxz;
    m.pxy = a1 - c1;
    m.pxz = a2 - c2;
    m.pyz = a3 - c3;
    m.mx = jx_xy - jx_xz;
    m.my = jy_yz - jy_xy;
    m.mz = jz_xz - jz_yz;
    return m;
}

// In: f[19] = offsets f_i - w_i, g[7] = energy populations.  Out: the
// post-collision values in the same representation.
template <typename T, int kForce>
__device__ __forceinline__ void collide(T f[19], T g[7], const Rates<T> &r)
{
    // ---- moments of the offsets (Eq. 20, rho V = sum e_i f_i) -------------
    const Moments<T> m = moments(f);
    const T drho = m.rho;                       // rho - 1
    const T rho = T(1) + drho;

    // ---- energy lattice: theta (Eq. 30); buoyancy G (Eq. 16, along +z) ---
    const T th = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6];
    const T Gz = kForce == 2 ? r.gbeta * (th - r.theta_ref) : T(0);

    // momentum of the equilibria: j, or j + rho G / 2 for Guo's scheme
    const T jx = m.jx, jy = m.jy;
    const T jz = kForce == 2 ? m.jz + T(0.5) * rho * Gz : m.jz;

    // ---- non-conserved moments of the offsets, minus the offsets of m^eq
    //      (Eq. 24 with rho_0 = 1, minus its value at rho = 1, j = 0) -------
    const T jxx = jx * jx, jyy = jy * jy, jzz = jz * jz;
    const T jj = jxx + jyy + jzz;
    const T p1 = T(2) * jxx - (jyy + jzz);
    const T p2 = jyy - jzz;

    // relaxed deviations divided by the row norms: k_* = s (m - m^eq)/|M_k|^2
    T k_e = r.e * (m.e - (T(-11) * drho + T(19) * jj));
    T k_eps = r.eps * (m.eps - (T(3) * drho - T(5.5) * jj));
    T k_qx = r.qx * (m.qx + T(2.0 / 3.0) * jx);
    T k_qy = r.qy * (m.qy + T(2.0 / 3.0) * jy);
    T k_qz = r.qz * (m.qz + T(2.0 / 3.0) * jz);
    T k_pxx = r.pxx * (m.pxx - p1);
    T k_pixx = r.pixx * (m.pixx + T(0.5) * p1);
    T k_pww = r.pww * (m.pww - p2);
    T k_piww = r.piww * (m.piww + T(0.5) * p2);
    T k_pxy = r.pxy * (m.pxy - jx * jy);
    T k_pyz = r.pyz * (m.pyz - jy * jz);
    T k_pxz = r.pxz * (m.pxz - jx * jz);
    T k_mx = r.mx * m.mx;
    T k_my = r.my * m.my;
    T k_mz = r.mz * m.mz;

    const T inv_rho = T(1) / rho;
    const T ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;

    // Per-direction force terms added after the back-transform: F_i of
    // Eqs. (15)-(17) (models 0, 1) as K (e_iz - u_z) w_i feq_poly, or for
    // Guo's scheme the momentum row's share e_iz rho G / |M_jz|^2.
    T k0 = T(0), kp = T(0), km = T(0), c0 = T(0), jrow = T(0);
    if constexpr (kForce == 2) {
        // Fbar_i = w_i rho G [3 (e_iz - u_z) + 9 (e_i . u) e_iz]; its moments
        // enter as - (1 - s_k/2) (M Fbar)_k.  The momentum row: s_j (j - rho u)
        // - (1 - s_j/2) rho G = -rho G for any s_j, i.e. f_i += e_iz rho G / 10.
        constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
        constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
        const T A = rho * Gz;
        T fb[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const T w = i == 0 ? T(1.0 / 3.0) : (i < 7 ? T(1.0 / 18.0) : T(1.0 / 36.0));
            const T eu = T(ex[i]) * ux + T(ey[i]) * uy + T(ez[i]) * uz;
            fb[i] = w * A * (T(3) * (T(ez[i]) - uz) + T(9) * eu * T(ez[i]));
        }
        const Moments<T> mf = moments(fb);
        k_e -= r.he * mf.e;
        k_eps -= r.heps * mf.eps;
        k_qx -= r.hqx * mf.qx;
        k_qy -= r.hqy * mf.qy;
        k_qz -= r.hqz * mf.qz;
        k_pxx -= r.hpxx * mf.pxx;
        k_pixx -= r.hpixx * mf.pixx;
        k_pww -= r.hpww * mf.pww;
        k_piww -= r.hpiww * mf.piww;
        k_pxy -= r.hpxy * mf.pxy;
        k_pyz -= r.hpyz * mf.pyz;
        k_pxz -= r.hpxz * mf.pxz;
        k_mx -= r.hmx * mf.mx;
        k_my -= r.hmy * mf.my;
        k_mz -= r.hmz * mf.mz;
        jrow = A * T(0.1);
    } else {
        // Eqs. (15)-(17): F_i = 3 G (e_iz - u_z) f^eq_i, f^eq_i = rho w_i feq_poly
        c0 = T(1) - T(1.5) * (ux * ux + uy * uy + uz * uz);
        const T K = kForce == 1 ? T(3) * r.gbeta * (th - r.theta_ref)
                                : T(3) * r.gbeta * (th - r.theta_ref) * rho;
        k0 = K * (-uz);          // e_z = 0
        kp = K * (T(1) - uz);    // e_z = +1
        km = K * (T(-1) - uz);   // e_z = -1
    }
    const T w0 = T(1.0 / 3.0), w1 = T(1.0 / 18.0), w2 = T(1.0 / 36.0);
    // force term of a direction with e_z = 0, +1, -1 and e . u = t
    auto F0 = [&](T w, T t) { return kForce == 2 ? T(0) : k0 * w * feq_poly(c0, t); };
    auto Fp = [&](T w, T t) { return kForce == 2 ? jrow : kp * w * feq_poly(c0, t); };
    auto Fm = [&](T w, T t) { return kForce == 2 ? -jrow : km * w * feq_poly(c0, t); };

    // ---- back-transform f* = f - M^T k + F ----------------------------------
    f[0] = f[0] - (T(-30) * k_e + T(12) * k_eps) + F0(w0, T(0));

    {
        const T C = T(-11) * k_e - T(4) * k_eps + T(2) * k_pxx - T(4) * k_pixx;
        const T O = T(-4) * k_qx;
        f[1] = f[1] - (C + O) + F0(w1, ux);
        f[2] = f[2] - (C - O) + F0(w1, -ux);
    }
    {
        const T C = T(-11) * k_e - T(4) * k_eps - k_pxx + T(2) * k_pixx + k_pww - T(2) * k_piww;
        const T O = T(-4) * k_qy;
        f[3] = f[3] - (C + O) + F0(w1, uy);
        f[4] = f[4] - (C - O) + F0(w1, -uy);
    }
    {
        const T C = T(-11) * k_e - T(4) * k_eps - k_pxx + T(2) * k_pixx - k_pww + T(2) * k_piww;
        const T O = T(-4) * k_qz;
        f[5] = f[5] - (C + O) + Fp(w1, uz);
        f[6] = f[6] - (C - O) + Fm(w1, -uz);
    }
    {   // xy diagonals: (sx, sy) = 7 (+,+), 8 (-,+), 9 (+,-), 10 (-,-)
        const T D = T(8) * k_e + k_eps + k_pxx + k_pixx + k_pww + k_piww;
        const T X = k_qx + k_mx, Y = k_qy - k_my, P = k_pxy;
        const T tp = ux + uy, tm = uy - ux;
        f[7] = f[7] - (D + X + Y + P) + F0(w2, tp);
        f[8] = f[8] - (D - X + Y - P) + F0(w2, tm);
        f[9] = f[9] - (D + X - Y - P) + F0(w2, -tm);
        f[10] = f[10] - (D - X - Y + P) + F0(w2, -tp);
    }
    {   // xz diagonals: (sx, sz) = 11 (+,+), 12 (-,+), 13 (+,-), 14 (-,-)
        const T D = T(8) * k_e + k_eps + k_pxx + k_pixx - k_pww - k_piww;
        const T X = k_qx - k_mx, Z = k_qz + k_mz, P = k_pxz;
        const T tp = ux + uz, tm = uz - ux;
        f[11] = f[11] - (D + X + Z + P) + Fp(w2, tp);
        f[12] = f[12] - (D - X + Z - P) + Fp(w2, tm);
        f[13] = f[13] - (D + X - Z - P) + Fm(w2, -tm);
        f[14] = f[14] - (D - X - Z + P) + Fm(w2, -tp);
    }
    {   // yz diagonals: (sy, sz) = 15 (+,+), 16 (-,+), 17 (+,-), 18 (-,-)
        const T D = T(8) * k_e + k_eps - T(2) * (k_pxx + k_pixx);
        const T Y = k_qy + k_my, Z = k_qz - k_mz, P = k_pyz;
        const T tp = uy + uz, tm = uz - uy;
        f[15] = f[15] - (D + Y + Z + P) + Fp(w2, tp);
        f[16] = f[16] - (D - Y + Z - P) + Fp(w2, tm);
        f[17] = f[17] - (D + Y - Z - P) + Fm(w2, -tm);
        f[18] = f[18] - (D - Y - Z + P) + Fm(w2, -tp);
    }

    // ---- D3Q7-MRT (Eqs. 29-35): g* = g - N^T k, k = Q (n - n^eq)/|N_k|^2 ----
    const T sg = g[1] + g[2] + g[3] + g[4] + g[5] + g[6];
    const T n1 = g[1] - g[2], n2 = g[3] - g[4], n3 = g[5] - g[6];
    const T n4 = T(6) * g[0] - sg;
    const T syy = g[3] + g[4], szz = g[5] + g[6];
    const T n5 = T(2) * (g[1] + g[2]) - syy - szz;
    const T n6 = syy - szz;
    const T d1 = n1 - ux * th, d2 = n2 - uy * th, d3 = n3 - uz * th;
    const T q1 = r.q11 * d1 + r.q12 * d2 + r.q13 * d3;
    const T q2 = r.q12 * d1 + r.q22 * d2 + r.q23 * d3;
    const T q3 = r.q13 * d1 + r.q23 * d2 + r.q33 * d3;
    const T q4 = r.t4 * (n4 - T(0.75) * th);
    const T q5 = r.t5 * n5;
    const T q6 = r.t6 * n6;
    g[0] = g[0] - T(6) * q4;
    {
        const T C = T(2) * q5 - q4;
        g[1] = g[1] - (C + q1);
        g[2] = g[2] - (C - q1);
    }
    {
        const T C = q6 - q5 - q4;
        g[3] = g[3] - (C + q2);
        g[4] = g[4] - (C - q2);
    }
    {
        const T C = -q6 - q5 - q4;
        g[5] = g[5] - (C + q3);
        g[6] = g[6] - (C - q3);
    }
}

}  // namespace lbmx
