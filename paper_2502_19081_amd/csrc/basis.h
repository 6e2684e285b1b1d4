// Radial and angular basis of the ACE-style model, shared by the kernels and
// by the host code that tabulates the Gaunt coefficients (so both use one
// spherical-harmonic convention).
#pragma once

#include "internal.h"

namespace mlmix {

// Chebyshev radial basis with the (1 - (r/rc)^2)^2 envelope and its
// derivative (T_n' = n U_{n-1}).
template <typename T>
__host__ __device__ inline void radial(int nrad, T r, T rc, T *R, T *dR)
{
    T inv = T(1) / rc;
    T x = T(2) * r * inv - T(1);
    T s = r * inv;
    T w = T(1) - s * s;
    T f = w * w;
    T df = T(-4) * s * w * inv;
    T t0 = T(1), t1 = x, u0 = T(1), u1 = T(2) * x;
#pragma unroll
    for (int k = 0; k < kMaxNrad; ++k) {
        if (k < nrad) {
            T tk, dtk;
            if (k == 0) {
                tk = T(1);
                dtk = T(0);
            } else if (k == 1) {
                tk = x;
                dtk = T(1);
            } else {
                tk = T(2) * x * t1 - t0;
                T uk1 = u1;  // U_{k-1}
                dtk = T(k) * uk1;
                t0 = t1;
                t1 = tk;
                T uk = T(2) * x * u1 - u0;
                u0 = u1;
                u1 = uk;
            }
            R[k] = tk * f;
            dR[k] = dtk * (T(2) * inv) * f + tk * df;
        }
    }
}

// 1/k for the small integers of the Legendre recurrence (k <= 2 lmax + 1).
template <typename T>
__host__ __device__ inline T inv_small(int k)
{
    switch (k) {
    case 1:
        return T(1.0);
    case 2:
        return T(0.5);
    case 3:
        return T(1.0 / 3.0);
    case 4:
        return T(0.25);
    case 5:
        return T(0.2);
    case 6:
        return T(1.0 / 6.0);
    case 7:
        return T(1.0 / 7.0);
    default:
        return T(1) / T(k);
    }
}

// Real orthonormal spherical harmonics of the unit vector (x, y, z) and their
// gradients with respect to (x, y, z) of the polynomial extension, streamed
// in (m, l) order: Y_lm = K_lm Q_l^|m|(z) {C_m, 1, S_|m|}, Q_l^m = d^m P_l/dz^m
// by the three-term recurrence, C_m + i S_m = (x + i y)^m, dQ_l^m/dz = Q_l^{m+1}.
// Only the orders m_lo <= |m| <= m_hi are emitted (the same values as the
// full stream gives for them).
template <typename T, typename F>
__host__ __device__ inline void ylm_stream(int lmax, T x, T y, T z, const T *__restrict__ K,
                                           F &&emit, int m_lo = 0, int m_hi = 1 << 30)
{
    T Cm = T(1), Sm = T(0), Cp = T(0), Sp = T(0);
    T dfm = T(1);
    const int mtop = m_hi < lmax ? m_hi : lmax;
    for (int m = 0; m <= mtop; ++m) {
        if (m > 0) {
            T c = x * Cm - y * Sm;
            T s = x * Sm + y * Cm;
            Cp = Cm;
            Sp = Sm;
            Cm = c;
            Sm = s;
            dfm *= T(2 * m - 1);
        }
        if (m < m_lo)
            continue;
        T dfm1 = dfm * T(2 * m + 1);
        T qa1 = T(0), qa2 = T(0), qb1 = T(0), qb2 = T(0);
        for (int l = m; l <= lmax; ++l) {
            T qa = (l == m) ? dfm
                            : (T(2 * l - 1) * z * qa1 - T(l + m - 1) * qa2) * inv_small<T>(l - m);
            T qb = (l == m) ? T(0)
                            : (l == m + 1 ? dfm1
                                          : (T(2 * l - 1) * z * qb1 - T(l + m) * qb2) *
                                                inv_small<T>(l - m - 1));
            int base = l * l + l;
            if (m == 0) {
                T k0 = K[base];
                emit(base, k0 * qa, T(0), T(0), k0 * qb);
            } else {
                T kp = K[base + m];
                T kq = kp * qa;
                T fm = T(m);
                emit(base + m, kq * Cm, kq * fm * Cp, -kq * fm * Sp, kp * qb * Cm);
                emit(base - m, kq * Sm, kq * fm * Sp, kq * fm * Cp, kp * qb * Sm);
            }
            qa2 = qa1;
            qa1 = qa;
            qb2 = qb1;
            qb1 = qb;
        }
    }
}

}  // namespace mlmix
