// Device quaternion and Lie-group helpers (Sec. 2.9 and Appendix A of
// arXiv:1903.12609).  Quaternions are double4 (x = q0 scalar part, y, z, w =
// q1, q2, q3); vectors are double3.
#pragma once
#include <hip/hip_runtime.h>

namespace fil {

struct V3 {
    double x, y, z;
};

__device__ __forceinline__ V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

struct Q4 {
    double w, x, y, z;  // (q0, q1, q2, q3)
};

// Hamilton product (p0 q0 - p.q, p0 q + q0 p + p x q)
__device__ __forceinline__ Q4 qmul(Q4 p, Q4 q) {
    return Q4{p.w * q.w - p.x * q.x - p.y * q.y - p.z * q.z,
              p.w * q.x + q.w * p.x + p.y * q.z - p.z * q.y,
              p.w * q.y + q.w * p.y + p.z * q.x - p.x * q.z,
              p.w * q.z + q.w * p.z + p.x * q.y - p.y * q.x};
}
__device__ __forceinline__ Q4 qconj(Q4 q) { return Q4{q.w, -q.x, -q.y, -q.z}; }

// Columns of the rotation matrix R(q): the material frame t = R e_x, mu = R e_y, nu = R e_z
__device__ __forceinline__ V3 frame_t(Q4 q) {
    return v3(1.0 - 2.0 * (q.y * q.y + q.z * q.z), 2.0 * (q.x * q.y + q.z * q.w), 2.0 * (q.x * q.z - q.y * q.w));
}
__device__ __forceinline__ V3 frame_mu(Q4 q) {
    return v3(2.0 * (q.x * q.y - q.z * q.w), 1.0 - 2.0 * (q.x * q.x + q.z * q.z), 2.0 * (q.z * q.y + q.x * q.w));
}
__device__ __forceinline__ V3 frame_nu(Q4 q) {
    return v3(2.0 * (q.x * q.z + q.y * q.w), 2.0 * (q.z * q.y - q.x * q.w), 1.0 - 2.0 * (q.y * q.y + q.x * q.x));
}
// R(q) v = t v_x + mu v_y + nu v_z
__device__ __forceinline__ V3 qrotate(Q4 q, V3 v) {
    return v.x * frame_t(q) + v.y * frame_mu(q) + v.z * frame_nu(q);
}

// Square root (Appendix A.1): (sqrt((p0+1)/2), p / sqrt(2(p0+1))), (0,0,0,1) at p0 = -1
__device__ __forceinline__ Q4 qsqrt(Q4 p) {
    if (p.w == -1.0) return Q4{0.0, 0.0, 0.0, 1.0};
    const double h = sqrt(0.5 * (p.w + 1.0));
    const double s = 0.5 / h;  // 1/sqrt(2(p0+1))
    return Q4{h, p.x * s, p.y * s, p.z * s};
}

// exp(u) = (cos(|u|/2), sin(|u|/2) u/|u|); sin(x/2)/x by its series below 1e-4
__device__ __forceinline__ Q4 qexp(V3 u) {
    const double x2 = dot(u, u);
    const double x = sqrt(x2);
    double s, c;
    sincos(0.5 * x, &s, &c);
    const double k = x < 1e-4 ? 0.5 - x2 / 48.0 : s / x;
    return Q4{c, k * u.x, k * u.y, k * u.z};
}

// dexp^{-1}_u(w) = w - u x w / 2 + k(|u|) u x (u x w),
// k(x) = (2 - x cot(x/2)) / (2 x^2), by its series 1/12 + x^2/720 + x^4/30240 below 1e-3
__device__ __forceinline__ V3 dexpinv(V3 u, V3 w) {
    const double x2 = dot(u, u);
    double k;
    if (x2 < 1e-6) {
        k = 1.0 / 12.0 + x2 * (1.0 / 720.0 + x2 * (1.0 / 30240.0));
    } else {
        const double x = sqrt(x2);
        double s, c;
        sincos(0.5 * x, &s, &c);
        k = (2.0 - x * c / s) / (2.0 * x2);
    }
    const V3 uw = cross(u, w);
    return w - 0.5 * uw + k * cross(u, uw);
}

// Discrete internal moment between segments n and n+1 (Sec. 2.9.2):
// M = R(h) D (2 [h^* . (q1 - q0)/dL]_{R^3} - kappa),  h = (q1 . q0^*)^{1/2} . q0,
// D = diag(KT, KB, KB)
__device__ __forceinline__ V3 joint_moment(Q4 q0, Q4 q1, V3 kap, double dL, double KB, double KT) {
    const Q4 h = qmul(qsqrt(qmul(q1, qconj(q0))), q0);
    const double idl = 2.0 / dL;
    const Q4 dq{(q1.w - q0.w) * idl, (q1.x - q0.x) * idl, (q1.y - q0.y) * idl, (q1.z - q0.z) * idl};
    const Q4 p = qmul(qconj(h), dq);
    const V3 z = v3(KT * (p.x - kap.x), KB * (p.y - kap.y), KB * (p.z - kap.z));
    return qrotate(h, z);
}

}  // namespace fil
