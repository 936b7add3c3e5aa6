// collide.hpp -- per-node double-MRT collision for the MI355X step kernel.
//
// Li, Yang & Zhang (arXiv:1511.04633), Sec. 3.  D3Q19 flow lattice with the
// moment basis of Eqs. (21)-(22), equilibrium moments of Eq. (24) (rho_0 = 1),
// diagonal relaxation S (Eqs. 23, 26), Boussinesq force of Eqs. (15)-(17)
// added after the collision (Eq. 14); D3Q7 energy lattice with N of Eq. (32),
// n^eq of Eq. (33) and a diagonal Q (Eqs. 35-36, isotropic diffusion).
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
    T t1, t2, t3, t4, t5, t6;   // energy moments n_1..n_6 (n_0 is conserved)
    T gbeta;                    // g beta per unit theta (buoyancy scale applied)
    T theta_ref;
};

// Equilibrium of Eq. (17) without the rho w_i factor: 1 + 3 t + 4.5 t^2 - 1.5 u.u,
// with c0 = 1 - 1.5 u.u and t = e_i . u.
template <typename T>
__device__ __forceinline__ T feq_poly(T c0, T t)
{
    return c0 + t * (T(3) + T(4.5) * t);
}

// In: f[19] = offsets f_i - w_i, g[7] = energy populations.  Out: the
// post-collision values in the same representation.  Also returns the
// node's density, velocity and temperature (pre-collision) on request.
template <typename T>
__device__ __forceinline__ void collide(T f[19], T g[7], const Rates<T> &r)
{
    // ---- pair sums and differences --------------------------------------
    const T Sx = f[1] + f[2], Dx = f[1] - f[2];
    const T Sy = f[3] + f[4], Dy = f[3] - f[4];
    const T Sz = f[5] + f[6], Dz = f[5] - f[6];
    // xy plane: 7 (+,+) <-> 10 (-,-), 8 (-,+) <-> 9 (+,-)
    const T a1 = f[7] + f[10], b1 = f[7] - f[10], c1 = f[8] + f[9], d1 = f[8] - f[9];
    // xz plane: 11 (+,+) <-> 14 (-,-), 12 (-,+) <-> 13 (+,-)
    const T a2 = f[11] + f[14], b2 = f[11] - f[14], c2 = f[12] + f[13], d2 = f[12] - f[13];
    // yz plane: 15 (+,+) <-> 18 (-,-), 16 (-,+) <-> 17 (+,-)
    const T a3 = f[15] + f[18], b3 = f[15] - f[18], c3 = f[16] + f[17], d3 = f[16] - f[17];

    const T sxy = a1 + c1, sxz = a2 + c2, syz = a3 + c3;
    const T jx_xy = b1 - d1, jy_xy = b1 + d1;
    const T jx_xz = b2 - d2, jz_xz = b2 + d2;
    const T jy_yz = b3 - d3, jz_yz = b3 + d3;

    const T s_ax = Sx + Sy + Sz;
    const T s_dg = sxy + sxz + syz;

    // ---- conserved moments (Eq. 20, rho V = sum e_i f_i) ----------------
    const T drho = f[0] + s_ax + s_dg;          // rho - 1
    const T jx = Dx + jx_xy + jx_xz;
    const T jy = Dy + jy_xy + jy_yz;
    const T jz = Dz + jz_xz + jz_yz;
    const T rho = T(1) + drho;

    // ---- non-conserved moments of the offsets, minus the offsets of m^eq
    //      (Eq. 24 with rho_0 = 1, minus its value at rho = 1, j = 0) -------
    const T jxx = jx * jx, jyy = jy * jy, jzz = jz * jz;
    const T jj = jxx + jyy + jzz;
    const T p1 = T(2) * jxx - (jyy + jzz);
    const T p2 = jyy - jzz;

    const T m_e = T(-30) * f[0] - T(11) * s_ax + T(8) * s_dg;
    const T m_eps = T(12) * f[0] - T(4) * s_ax + s_dg;
    const T m_qx = T(-4) * Dx + jx_xy + jx_xz;
    const T m_qy = T(-4) * Dy + jy_xy + jy_yz;
    const T m_qz = T(-4) * Dz + jz_xz + jz_yz;
    const T m_pxx = T(2) * Sx - Sy - Sz + sxy + sxz - T(2) * syz;
    const T m_pixx = T(-4) * Sx + T(2) * (Sy + Sz) + sxy + sxz - T(2) * syz;
    const T m_pww = Sy - Sz + sxy - sxz;
    const T m_piww = T(2) * (Sz - Sy) + sxy - sxz;
    const T m_pxy = a1 - c1;
    const T m_pxz = a2 - c2;
    const T m_pyz = a3 - c3;
    const T m_mx = jx_xy - jx_xz;
    const T m_my = jy_yz - jy_xy;
    const T m_mz = jz_xz - jz_yz;

    // relaxed deviations divided by the row norms: k_* = s (m - m^eq)/|M_k|^2
    const T k_e = r.e * (m_e - (T(-11) * drho + T(19) * jj));
    const T k_eps = r.eps * (m_eps - (T(3) * drho - T(5.5) * jj));
    const T k_qx = r.qx * (m_qx + T(2.0 / 3.0) * jx);
    const T k_qy = r.qy * (m_qy + T(2.0 / 3.0) * jy);
    const T k_qz = r.qz * (m_qz + T(2.0 / 3.0) * jz);
    const T k_pxx = r.pxx * (m_pxx - p1);
    const T k_pixx = r.pixx * (m_pixx + T(0.5) * p1);
    const T k_pww = r.pww * (m_pww - p2);
    const T k_piww = r.piww * (m_piww + T(0.5) * p2);
    const T k_pxy = r.pxy * (m_pxy - jx * jy);
    const T k_pyz = r.pyz * (m_pyz - jy * jz);
    const T k_pxz = r.pxz * (m_pxz - jx * jz);
    const T k_mx = r.mx * m_mx;
    const T k_my = r.my * m_my;
    const T k_mz = r.mz * m_mz;

    // ---- energy lattice: theta (Eq. 30) before f is overwritten ---------
    const T th = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6];

    // ---- Boussinesq force, Eqs. (15)-(17): F_i = 3 G (e_iz - u_z) f^eq_i,
    //      G = g beta (theta - theta_ref) along +z ----------------------------
    const T inv_rho = T(1) / rho;
    const T ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    const T c0 = T(1) - T(1.5) * (ux * ux + uy * uy + uz * uz);
    const T K = T(3) * r.gbeta * (th - r.theta_ref) * rho;
    const T k0 = K * (-uz);          // e_z = 0
    const T kp = K * (T(1) - uz);    // e_z = +1
    const T km = K * (T(-1) - uz);   // e_z = -1
    const T w0 = T(1.0 / 3.0), w1 = T(1.0 / 18.0), w2 = T(1.0 / 36.0);

    // ---- back-transform f* = f - M^T k + F ----------------------------------
    f[0] = f[0] - (T(-30) * k_e + T(12) * k_eps) + k0 * w0 * c0;

    {
        const T C = T(-11) * k_e - T(4) * k_eps + T(2) * k_pxx - T(4) * k_pixx;
        const T O = T(-4) * k_qx;
        const T F0 = k0 * w1;
        f[1] = f[1] - (C + O) + F0 * feq_poly(c0, ux);
        f[2] = f[2] - (C - O) + F0 * feq_poly(c0, -ux);
    }
    {
        const T C = T(-11) * k_e - T(4) * k_eps - k_pxx + T(2) * k_pixx + k_pww - T(2) * k_piww;
        const T O = T(-4) * k_qy;
        const T F0 = k0 * w1;
        f[3] = f[3] - (C + O) + F0 * feq_poly(c0, uy);
        f[4] = f[4] - (C - O) + F0 * feq_poly(c0, -uy);
    }
    {
        const T C = T(-11) * k_e - T(4) * k_eps - k_pxx + T(2) * k_pixx - k_pww + T(2) * k_piww;
        const T O = T(-4) * k_qz;
        f[5] = f[5] - (C + O) + kp * w1 * feq_poly(c0, uz);
        f[6] = f[6] - (C - O) + km * w1 * feq_poly(c0, -uz);
    }
    {   // xy diagonals: (sx, sy) = 7 (+,+), 8 (-,+), 9 (+,-), 10 (-,-)
        const T D = T(8) * k_e + k_eps + k_pxx + k_pixx + k_pww + k_piww;
        const T X = k_qx + k_mx, Y = k_qy - k_my, P = k_pxy;
        const T F0 = k0 * w2;
        const T tp = ux + uy, tm = uy - ux;
        f[7] = f[7] - (D + X + Y + P) + F0 * feq_poly(c0, tp);
        f[8] = f[8] - (D - X + Y - P) + F0 * feq_poly(c0, tm);
        f[9] = f[9] - (D + X - Y - P) + F0 * feq_poly(c0, -tm);
        f[10] = f[10] - (D - X - Y + P) + F0 * feq_poly(c0, -tp);
    }
    {   // xz diagonals: (sx, sz) = 11 (+,+), 12 (-,+), 13 (+,-), 14 (-,-)
        const T D = T(8) * k_e + k_eps + k_pxx + k_pixx - k_pww - k_piww;
        const T X = k_qx - k_mx, Z = k_qz + k_mz, P = k_pxz;
        const T Fp = kp * w2, Fm = km * w2;
        const T tp = ux + uz, tm = uz - ux;
        f[11] = f[11] - (D + X + Z + P) + Fp * feq_poly(c0, tp);
        f[12] = f[12] - (D - X + Z - P) + Fp * feq_poly(c0, tm);
        f[13] = f[13] - (D + X - Z - P) + Fm * feq_poly(c0, -tm);
        f[14] = f[14] - (D - X - Z + P) + Fm * feq_poly(c0, -tp);
    }
    {   // yz diagonals: (sy, sz) = 15 (+,+), 16 (-,+), 17 (+,-), 18 (-,-)
        const T D = T(8) * k_e + k_eps - T(2) * (k_pxx + k_pixx);
        const T Y = k_qy + k_my, Z = k_qz - k_mz, P = k_pyz;
        const T Fp = kp * w2, Fm = km * w2;
        const T tp = uy + uz, tm = uz - uy;
        f[15] = f[15] - (D + Y + Z + P) + Fp * feq_poly(c0, tp);
        f[16] = f[16] - (D - Y + Z - P) + Fp * feq_poly(c0, tm);
        f[17] = f[17] - (D + Y - Z - P) + Fm * feq_poly(c0, -tm);
        f[18] = f[18] - (D - Y - Z + P) + Fm * feq_poly(c0, -tp);
    }

    // ---- D3Q7-MRT (Eqs. 29-35): g* = g - N^T k, k = Q (n - n^eq)/|N_k|^2 ----
    const T sg = g[1] + g[2] + g[3] + g[4] + g[5] + g[6];
    const T n1 = g[1] - g[2], n2 = g[3] - g[4], n3 = g[5] - g[6];
    const T n4 = T(6) * g[0] - sg;
    const T syy = g[3] + g[4], szz = g[5] + g[6];
    const T n5 = T(2) * (g[1] + g[2]) - syy - szz;
    const T n6 = syy - szz;
    const T q1 = r.t1 * (n1 - ux * th);
    const T q2 = r.t2 * (n2 - uy * th);
    const T q3 = r.t3 * (n3 - uz * th);
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
