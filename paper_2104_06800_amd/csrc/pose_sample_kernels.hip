// The paper's pose M-step by Monte-Carlo P3P sampling on gfx950 (VOLDOR+SLAM sec. III-A
// "Uncertainty-aware Pose Estimation", its sampling equation), one frame per launch pair:
//
//   samples : one thread per sample.  Three pixels drawn with probability proportional to the
//             rigidness posterior q_t (Philox draw of a pixel, accepted when a second draw is
//             below q_t and the pixel has a depth and an observation; a bounded number of
//             attempts per point), their 3D points x~/rho and the unit bearings of their
//             observations o_t = p_{t-1} + X_t(p_{t-1}) in frame t; P3P from the law of
//             cosines of the three rays (Grunert's elimination to a quartic in the ratio of two
//             ray lengths, real roots bracketed between the critical points and refined by
//             safeguarded Newton steps, then Newton on the three cosine equations); of its
//             solutions the one nearest the frame's current pose in the kernel metric; the
//             rigid motion from the three point pairs by orthonormal triads.  All in FP64 (a
//             few thousand evaluations per frame).
//   mode    : one block.  Meanshift with the Gaussian kernel in the left-update chart from the
//             current pose, block sums in a fixed order; then the covariance of the samples
//             about the mode by iterated 3-sigma inlier fits (covariance divided by the
//             Gaussian truncation factor, eigenvalues floored by a one-thread Jacobi
//             eigen-decomposition).  The frame's pose becomes the mode.
#include "device.h"
#include "kernels.h"

namespace vd {

namespace {

constexpr int kPsBlock = 256;

// P(chi2_8 <= 9) / P(chi2_6 <= 9): the share of a 6-D Gaussian's variance inside 3 sigma
__device__ __forceinline__ double trunc_kappa() {
    const double e = exp(-4.5);
    return (1.0 - e * (1.0 + 4.5 + 10.125 + 15.1875)) / (1.0 - e * (1.0 + 4.5 + 10.125));
}

__device__ inline double poly_eval(const double* c, int deg, double x) {
    double r = c[deg];
    for (int i = deg - 1; i >= 0; --i) r = r * x + c[i];
    return r;
}

// real roots of the polynomial c[0] + c[1] x + ... + c[deg] x^deg (deg <= 4, c[deg] != 0),
// sorted; double roots that touch zero without a sign change are not reported
__device__ int real_roots(const double* c, int deg, double* out) {
    if (deg == 1) { out[0] = -c[0] / c[1]; return 1; }
    if (deg == 2) {
        const double a = c[2], b = c[1], cc = c[0];
        const double disc = b * b - 4.0 * a * cc;
        if (disc < 0.0) return 0;
        const double sq = sqrt(disc);
        const double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
        if (q == 0.0) { out[0] = 0.0; return 1; }
        double r0 = q / a, r1 = cc / q;
        if (r0 > r1) { const double tmp = r0; r0 = r1; r1 = tmp; }
        out[0] = r0; out[1] = r1;
        return 2;
    }
    // critical points from the derivative, then one sign change per bracket
    double d[4];
    for (int i = 1; i <= deg; ++i) d[i - 1] = i * c[i];
    double crit[3];
    const int nc = real_roots(d, deg - 1, crit);
    double bound = 0.0;
    for (int i = 0; i < deg; ++i) bound = fmax(bound, fabs(c[i] / c[deg]));
    bound += 1.0;
    double pts[5];
    int np = 0;
    pts[np++] = -bound;
    for (int i = 0; i < nc; ++i) pts[np++] = fmin(fmax(crit[i], -bound), bound);
    pts[np++] = bound;
    int n = 0;
    for (int k = 0; k + 1 < np; ++k) {
        double lo = pts[k], hi = pts[k + 1];
        double flo = poly_eval(c, deg, lo), fhi = poly_eval(c, deg, hi);
        if (flo == 0.0) { out[n++] = lo; continue; }
        if ((flo < 0.0) == (fhi < 0.0)) continue;
        double x = 0.5 * (lo + hi);
        for (int it = 0; it < 100; ++it) {
            const double fx = poly_eval(c, deg, x);
            if (fx == 0.0) break;
            if ((fx < 0.0) == (flo < 0.0)) lo = x; else hi = x;
            const double dfx = poly_eval(d, deg - 1, x);
            double xn = dfx != 0.0 ? x - fx / dfx : 0.5 * (lo + hi);
            if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
            if (fabs(xn - x) <= 1e-15 * fabs(x) || hi - lo <= 1e-15 * fmax(fabs(lo), fabs(hi))) { x = xn; break; }
            x = xn;
        }
        out[n++] = x;
    }
    return n;
}

__device__ inline void poly_mul(const double* a, int da, const double* b, int db, double* out) {
    for (int i = 0; i <= da + db; ++i) out[i] = 0.0;
    for (int i = 0; i <= da; ++i)
        for (int j = 0; j <= db; ++j) out[i + j] += a[i] * b[j];
}

__device__ inline void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// orthonormal frame (columns e1, e3 x e1, e3) of the triangle Y[0..2]
__device__ inline bool triad(const double Y[3][3], double T[9]) {
    double e1[3], e2[3], e3[3], v[3], w[3];
    for (int i = 0; i < 3; ++i) { v[i] = Y[1][i] - Y[0][i]; w[i] = Y[2][i] - Y[0][i]; }
    const double n1 = sqrt(dot3(v, v));
    cross3(v, w, e3);
    const double n3 = sqrt(dot3(e3, e3));
    if (!(n1 > 0.0) || !(n3 > 0.0)) return false;
    for (int i = 0; i < 3; ++i) { e1[i] = v[i] / n1; e3[i] = e3[i] / n3; }
    cross3(e3, e1, e2);
    for (int i = 0; i < 3; ++i) { T[3 * i + 0] = e1[i]; T[3 * i + 1] = e2[i]; T[3 * i + 2] = e3[i]; }
    return true;
}

// chart coordinates (w, v) of (R, t) about (Rm, tm): w = log(R Rm^T), v = t - R Rm^T tm
__device__ inline void chart_d(const double* R, const double* t, const double* Rm, const double* tm, double* d) {
    double dR[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            dR[3 * i + j] = R[3 * i + 0] * Rm[3 * j + 0] + R[3 * i + 1] * Rm[3 * j + 1] + R[3 * i + 2] * Rm[3 * j + 2];
    log_so3(dR, d);
    for (int i = 0; i < 3; ++i) d[3 + i] = t[i] - (dR[3 * i] * tm[0] + dR[3 * i + 1] * tm[1] + dR[3 * i + 2] * tm[2]);
}

struct PsFrame {
    double Rc[9], tc[3];      // current pose of frame t
    double Rp[9], tp[3];      // pose of frame t - 1 (t >= 2)
    double kinv[6];           // inverse kernel variances
};

__device__ inline void frame_setup(const PoseSampleArgs& a, const double* pose, int t, PsFrame& F) {
    exp_so3(pose + 6 * (t - 1), F.Rc);
    for (int i = 0; i < 3; ++i) F.tc[i] = pose[6 * (t - 1) + 3 + i];
    if (t >= 2) {
        exp_so3(pose + 6 * (t - 2), F.Rp);
        for (int i = 0; i < 3; ++i) F.tp[i] = pose[6 * (t - 2) + 3 + i];
    }
    const double tn = sqrt(dot3(F.tc, F.tc));
    const double sv = a.sigma_t_rel * fmax(tn, 1e-12);
    for (int i = 0; i < 3; ++i) { F.kinv[i] = 1.0 / (a.sigma_w * a.sigma_w); F.kinv[3 + i] = 1.0 / (sv * sv); }
}

// unit bearing of pixel j's observation in frame t (FP64); false where it does not exist
__device__ bool observation(const PoseSampleArgs& a, const PoseSampleBufs& B, const PsFrame& F, int t, int j,
                            double* f, double* X) {
    const int v = j / a.W, u = j - v * a.W;
    const float rf = B.idepth[j];
    if (!(rf > 0.f) || !isfinite(rf)) return false;
    const double rho = (double)rf;
    const double x0 = ((double)u - a.cx) / a.fx, x1 = ((double)v - a.cy) / a.fy;
    double px, py, X0, X1;
    const size_t plane = (size_t)a.H * a.W;
    if (t == 1) {
        px = u; py = v;
        const float2 fl = B.flow[j];
        if (!isfinite(fl.x) || !isfinite(fl.y)) return false;
        X0 = fl.x; X1 = fl.y;
    } else {
        const double qx = F.Rp[0] * x0 + F.Rp[1] * x1 + F.Rp[2] + rho * F.tp[0];
        const double qy = F.Rp[3] * x0 + F.Rp[4] * x1 + F.Rp[5] + rho * F.tp[1];
        const double qz = F.Rp[6] * x0 + F.Rp[7] * x1 + F.Rp[8] + rho * F.tp[2];
        if (!(qz > 0.0)) return false;
        px = a.fx * qx / qz + a.cx;
        py = a.fy * qy / qz + a.cy;
        if (!(px >= 0.0 && px <= (double)(a.W - 1) && py >= 0.0 && py <= (double)(a.H - 1))) return false;
        const int ix = (int)floor(px), iy = (int)floor(py);
        const int ix1 = min(ix + 1, a.W - 1), iy1 = min(iy + 1, a.H - 1);
        const double ax = px - ix, ay = py - iy;
        const float2* fl = B.flow + (size_t)(t - 1) * plane;
        const float2 f00 = fl[iy * a.W + ix], f01 = fl[iy * a.W + ix1], f10 = fl[iy1 * a.W + ix], f11 = fl[iy1 * a.W + ix1];
        if (!isfinite(f00.x) || !isfinite(f00.y) || !isfinite(f01.x) || !isfinite(f01.y) || !isfinite(f10.x) ||
            !isfinite(f10.y) || !isfinite(f11.x) || !isfinite(f11.y))
            return false;
        X0 = (1.0 - ay) * ((1.0 - ax) * f00.x + ax * f01.x) + ay * ((1.0 - ax) * f10.x + ax * f11.x);
        X1 = (1.0 - ay) * ((1.0 - ax) * f00.y + ax * f01.y) + ay * ((1.0 - ax) * f10.y + ax * f11.y);
    }
    const double bx = (px + X0 - a.cx) / a.fx, by = (py + X1 - a.cy) / a.fy;
    const double n = sqrt(bx * bx + by * by + 1.0);
    if (!isfinite(n)) return false;
    f[0] = bx / n; f[1] = by / n; f[2] = 1.0 / n;
    X[0] = x0 / rho; X[1] = x1 / rho; X[2] = 1.0 / rho;
    return true;
}

// the P3P solution of (X, f) nearest (Rc, tc) in the kernel metric; false if none
__device__ bool p3p_nearest(const double X[3][3], const double f[3][3], const PsFrame& F, double* Rb, double* tb) {
    double d01[3], d02[3], d12[3];
    for (int i = 0; i < 3; ++i) { d12[i] = X[1][i] - X[2][i]; d02[i] = X[0][i] - X[2][i]; d01[i] = X[0][i] - X[1][i]; }
    const double a2 = dot3(d12, d12), b2 = dot3(d02, d02), c2 = dot3(d01, d01);
    const double ca = dot3(f[1], f[2]), cb = dot3(f[0], f[2]), cg = dot3(f[0], f[1]);
    // u = Nu(v) / Du(v) from the difference of two cosine laws; the second times Du^2: quartic
    const double Nu[3] = {a2 - c2 + b2, -2.0 * (a2 - c2) * cb, a2 - c2 - b2};
    const double Du[2] = {2.0 * b2 * cg, -2.0 * b2 * ca};
    double DD[3], NN[5], ND[4], L[5], Q[5];
    poly_mul(Du, 1, Du, 1, DD);
    poly_mul(Nu, 2, Nu, 2, NN);
    poly_mul(Nu, 2, Du, 1, ND);
    const double cosv[3] = {1.0, -2.0 * cb, 1.0};
    poly_mul(cosv, 2, DD, 2, L);
    for (int i = 0; i < 5; ++i) {
        const double lhs = b2 * ((i < 3 ? DD[i] : 0.0) + NN[i] - 2.0 * cg * (i < 4 ? ND[i] : 0.0));
        Q[i] = lhs - c2 * L[i];
    }
    int deg = 4;
    double mx = 0.0;
    for (int i = 0; i < 5; ++i) mx = fmax(mx, fabs(Q[i]));
    if (!(mx > 0.0) || !isfinite(mx)) return false;
    while (deg > 0 && Q[deg] == 0.0) --deg;
    if (deg == 0) return false;
    double roots[4];
    const int nr = real_roots(Q, deg, roots);
    double dQ[4];
    for (int i = 1; i <= deg; ++i) dQ[i - 1] = i * Q[i];
    bool found = false;
    double bestd = 0.0;
    for (int k = 0; k < nr; ++k) {
        double v = roots[k];
        for (int it = 0; it < 3; ++it) {
            const double dv = poly_eval(dQ, deg - 1, v);
            if (dv == 0.0) break;
            v = v - poly_eval(Q, deg, v) / dv;
        }
        const double du = Du[0] + Du[1] * v;
        if (!(v > 0.0) || du == 0.0) continue;
        const double u = (Nu[0] + Nu[1] * v + Nu[2] * v * v) / du;
        const double den = 1.0 + v * v - 2.0 * v * cb;
        if (!(u > 0.0) || !(den > 0.0)) continue;
        const double s1 = sqrt(b2 / den);
        double s[3] = {s1, u * s1, v * s1};
        for (int it = 0; it < 2; ++it) {
            const double F0 = s[1] * s[1] + s[2] * s[2] - 2.0 * s[1] * s[2] * ca - a2;
            const double F1 = s[0] * s[0] + s[2] * s[2] - 2.0 * s[0] * s[2] * cb - b2;
            const double F2 = s[0] * s[0] + s[1] * s[1] - 2.0 * s[0] * s[1] * cg - c2;
            const double J[9] = {0.0, 2.0 * s[1] - 2.0 * s[2] * ca, 2.0 * s[2] - 2.0 * s[1] * ca,
                                 2.0 * s[0] - 2.0 * s[2] * cb, 0.0, 2.0 * s[2] - 2.0 * s[0] * cb,
                                 2.0 * s[0] - 2.0 * s[1] * cg, 2.0 * s[1] - 2.0 * s[0] * cg, 0.0};
            // Cramer: J ds = F
            const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                               J[2] * (J[3] * J[7] - J[4] * J[6]);
            if (!(fabs(det) >= 1e-300)) break;
            const double Fv[3] = {F0, F1, F2};
            double ds[3];
            for (int c = 0; c < 3; ++c) {
                double M[9];
                for (int r = 0; r < 3; ++r)
                    for (int q = 0; q < 3; ++q) M[3 * r + q] = q == c ? Fv[r] : J[3 * r + q];
                ds[c] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                         M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
            }
            for (int c = 0; c < 3; ++c) s[c] -= ds[c];
        }
        if (!(s[0] > 0.0 && s[1] > 0.0 && s[2] > 0.0)) continue;
        double C[3][3];
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) C[i][c] = s[i] * f[i][c];
        double TC[9], TX[9], R[9], t[3];
        if (!triad(C, TC) || !triad(X, TX)) continue;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[3 * i + j] = TC[3 * i] * TX[3 * j] + TC[3 * i + 1] * TX[3 * j + 1] + TC[3 * i + 2] * TX[3 * j + 2];
        for (int i = 0; i < 3; ++i) t[i] = C[0][i] - (R[3 * i] * X[0][0] + R[3 * i + 1] * X[0][1] + R[3 * i + 2] * X[0][2]);
        double d[6];
        chart_d(R, t, F.Rc, F.tc, d);
        double m = 0.0;
        for (int i = 0; i < 6; ++i) m += d[i] * d[i] * F.kinv[i];
        if (!isfinite(m)) continue;
        if (!found || m < bestd) {
            found = true;
            bestd = m;
            for (int i = 0; i < 9; ++i) Rb[i] = R[i];
            for (int i = 0; i < 3; ++i) tb[i] = t[i];
        }
    }
    return found;
}

// cyclic Jacobi eigen-decomposition of a symmetric 6x6 matrix A (row-major, destroyed):
// eigenvalues in lam, eigenvectors in the columns of V
__device__ void jacobi6(double* A, double* lam, double* V) {
    for (int i = 0; i < 36; ++i) V[i] = (i % 7 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                tot += A[6 * i + j] * A[6 * i + j];
                if (i != j) off += A[6 * i + j] * A[6 * i + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < 5; ++p)
            for (int q = p + 1; q < 6; ++q) {
                const double apq = A[6 * p + q];
                if (apq == 0.0) continue;
                const double th = (A[6 * q + q] - A[6 * p + p]) / (2.0 * apq);
                const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                for (int k = 0; k < 6; ++k) {
                    const double akp = A[6 * k + p], akq = A[6 * k + q];
                    A[6 * k + p] = c * akp - s * akq;
                    A[6 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 6; ++k) {
                    const double apk = A[6 * p + k], aqk = A[6 * q + k];
                    A[6 * p + k] = c * apk - s * aqk;
                    A[6 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 6; ++k) {
                    const double vkp = V[6 * k + p], vkq = V[6 * k + q];
                    V[6 * k + p] = c * vkp - s * vkq;
                    V[6 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 6; ++i) lam[i] = A[7 * i];
}

// block sum of n doubles per thread (fixed order: wave trees, then the waves in order)
template <int NV>
__device__ void block_sum(double* v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[wid * NV + k] = x;
    }
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < kPsBlock / 64; ++w) s += red[w * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(64)
k_ps_samples(PoseSampleArgs a, PoseSampleBufs B, int t) {
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= a.S) return;
    PsFrame F;
    frame_setup(a, B.pose, t, F);
    const int npix = a.H * a.W;
    const size_t plane = (size_t)npix;
    const float* q = B.rigid + (size_t)(t - 1) * plane;
    const uint32_t word2 = ((uint32_t)a.it << 8) | ((uint32_t)t << 4) | 2u;
    double X[3][3], f[3][3];
    bool ok = true;
    for (int k = 0; k < 3 && ok; ++k) {
        bool got = false;
        for (int r = 0; r < a.tries && !got; ++r) {
            const uint4 x = philox10(make_uint4((uint32_t)g, (uint32_t)(k * a.tries + r), word2, a.window_id),
                                     a.key0, a.key1);
            const int j = (int)(((uint64_t)x.x * (uint64_t)npix) >> 32);
            const float uu = unit24(x.y);
            if (!(uu < q[j])) continue;
            got = observation(a, B, F, t, j, f[k], X[k]);
        }
        ok = got;
    }
    double* out = B.samples + (size_t)g * 12;
    double R[9], tt[3];
    if (ok) ok = p3p_nearest(X, f, F, R, tt);
    if (!ok) {
        for (int i = 0; i < 12; ++i) out[i] = __builtin_nan("");
        return;
    }
    for (int i = 0; i < 9; ++i) out[i] = R[i];
    for (int i = 0; i < 3; ++i) out[9 + i] = tt[i];
}

__global__ void __launch_bounds__(kPsBlock)
k_ps_mode(PoseSampleArgs a, PoseSampleBufs B, int t) {
    __shared__ double red[(kPsBlock / 64) * 22];
    __shared__ double mode_s[12];        // mode as R (9), t (3)
    __shared__ double mode_v[6];         // mode as a 6-vector
    __shared__ double sig_s[36], siginv_s[36], mu_s[6];
    __shared__ int flag_s, stop_s;
    const int tid = threadIdx.x;
    PsFrame F;
    frame_setup(a, B.pose, t, F);
    constexpr int PER = (4096 + kPsBlock - 1) / kPsBlock;   // samples per thread (S <= 4096)
    // count valid samples
    double cnt[1] = {0.0};
    for (int g = tid; g < a.S; g += kPsBlock) cnt[0] += isfinite(B.samples[(size_t)g * 12]) ? 1.0 : 0.0;
    block_sum<1>(cnt, red);
    const int valid = (int)cnt[0];
    double* cov = B.cov ? B.cov + 36 * (size_t)(t - 1) : nullptr;
    double* info = B.info ? B.info + 4 * (size_t)(t - 1) : nullptr;
    if (valid == 0) {
        if (tid < 36 && cov) cov[tid] = (tid % 7 == 0) ? 1.0 / F.kinv[tid / 7] : 0.0;
        if (tid < 4 && info) info[tid] = 0.0;
        return;
    }
    if (tid == 0) {
        for (int i = 0; i < 9; ++i) mode_s[i] = F.Rc[i];
        for (int i = 0; i < 3; ++i) mode_s[9 + i] = F.tc[i];
        for (int i = 0; i < 6; ++i) mode_v[i] = B.pose[6 * (t - 1) + i];
    }
    __syncthreads();
    // ---- meanshift
    int steps = 0;
    for (int step = 1; step <= 100; ++step) {
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int g = tid; g < a.S; g += kPsBlock) {
            const double* s = B.samples + (size_t)g * 12;
            if (!isfinite(s[0])) continue;
            double d[6];
            chart_d(s, s + 9, mode_s, mode_s + 9, d);
            double m = 0.0;
            for (int i = 0; i < 6; ++i) m += d[i] * d[i] * F.kinv[i];
            const double w = exp(-0.5 * m);
            acc[0] += w;
            for (int i = 0; i < 6; ++i) acc[1 + i] += w * d[i];
        }
        block_sum<7>(acc, red);
        steps = step;
        if (tid == 0) {
            stop_s = 0;
            if (acc[0] == 0.0) {
                stop_s = 1;
            } else {
                double delta[6], m = 0.0;
                for (int i = 0; i < 6; ++i) { delta[i] = acc[1 + i] / acc[0]; m += delta[i] * delta[i] * F.kinv[i]; }
                // mode <- left update by delta, kept both as (R, t) and as a 6-vector
                double E[9], R2[9], t2[3];
                exp_so3(delta, E);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        R2[3 * i + j] = E[3 * i] * mode_s[j] + E[3 * i + 1] * mode_s[3 + j] + E[3 * i + 2] * mode_s[6 + j];
                for (int i = 0; i < 3; ++i)
                    t2[i] = E[3 * i] * mode_s[9] + E[3 * i + 1] * mode_s[10] + E[3 * i + 2] * mode_s[11] + delta[3 + i];
                double w[3];
                log_so3(R2, w);
                for (int i = 0; i < 3; ++i) { mode_v[i] = w[i]; mode_v[3 + i] = t2[i]; }
                // the (R, t) form is rebuilt from the 6-vector, as the next step's chart uses it
                exp_so3(mode_v, mode_s);
                for (int i = 0; i < 3; ++i) mode_s[9 + i] = t2[i];
                if (sqrt(m) < 1e-12) stop_s = 1;
            }
        }
        __syncthreads();
        if (stop_s) break;
    }
    // ---- covariance about the mode: iterated 3-sigma fits
    double dl[PER][6];
    bool inl[PER];
    for (int k = 0; k < PER; ++k) {
        const int g = tid + k * kPsBlock;
        inl[k] = false;
        if (g < a.S && isfinite(B.samples[(size_t)g * 12])) chart_d(B.samples + (size_t)g * 12, B.samples + (size_t)g * 12 + 9,
                                                                    mode_s, mode_s + 9, dl[k]);
        else for (int i = 0; i < 6; ++i) dl[k][i] = __builtin_nan("");
    }
    if (tid < 36) {
        sig_s[tid] = (tid % 7 == 0) ? 1.0 / F.kinv[tid / 7] : 0.0;
        siginv_s[tid] = (tid % 7 == 0) ? F.kinv[tid / 7] : 0.0;
    }
    if (tid < 6) mu_s[tid] = 0.0;
    __syncthreads();
    int n_in = 0, rounds = 0;
    const double kappa = trunc_kappa();
    for (int r = 1; r <= 20; ++r) {
        rounds = r;
        double c2[2] = {0.0, 0.0};      // inliers, changed
        bool nin[PER];
        for (int k = 0; k < PER; ++k) {
            nin[k] = false;
            if (!isfinite(dl[k][0])) continue;
            double e[6];
            for (int i = 0; i < 6; ++i) e[i] = dl[k][i] - mu_s[i];
            double m2 = 0.0;
            for (int i = 0; i < 6; ++i) {
                double row = 0.0;
                for (int j = 0; j < 6; ++j) row += siginv_s[6 * i + j] * e[j];
                m2 += e[i] * row;
            }
            nin[k] = m2 <= 9.0;
            c2[0] += nin[k] ? 1.0 : 0.0;
            c2[1] += (r > 1 && nin[k] != inl[k]) ? 1.0 : 0.0;
        }
        block_sum<2>(c2, red);
        if (c2[0] < 7.0 || (r > 1 && c2[1] == 0.0)) break;
        n_in = (int)c2[0];
        for (int k = 0; k < PER; ++k) inl[k] = nin[k];
        double mu[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < PER; ++k)
            if (inl[k]) for (int i = 0; i < 6; ++i) mu[i] += dl[k][i];
        block_sum<6>(mu, red);
        for (int i = 0; i < 6; ++i) mu[i] /= (double)n_in;
        double C[21];
        for (int i = 0; i < 21; ++i) C[i] = 0.0;
        for (int k = 0; k < PER; ++k) {
            if (!inl[k]) continue;
            double e[6];
            for (int i = 0; i < 6; ++i) e[i] = dl[k][i] - mu[i];
            int idx = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = i; j < 6; ++j) C[idx++] += e[i] * e[j];
        }
        block_sum<21>(C, red);
        if (tid == 0) {
            double A[36], lam[6], V[36];
            int idx = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = i; j < 6; ++j) {
                    A[6 * i + j] = A[6 * j + i] = C[idx++] / (double)n_in / kappa;
                }
            jacobi6(A, lam, V);
            for (int i = 0; i < 6; ++i) lam[i] = fmax(lam[i], a.eps);
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) {
                    double s = 0.0, si = 0.0;
                    for (int k = 0; k < 6; ++k) {
                        s += V[6 * i + k] * lam[k] * V[6 * j + k];
                        si += V[6 * i + k] / lam[k] * V[6 * j + k];
                    }
                    sig_s[6 * i + j] = s;
                    siginv_s[6 * i + j] = si;
                }
            for (int i = 0; i < 6; ++i) mu_s[i] = mu[i];
        }
        __syncthreads();
    }
    if (tid < 36 && cov) cov[tid] = sig_s[tid];
    if (tid == 0) {
        for (int i = 0; i < 6; ++i) B.pose[6 * (t - 1) + i] = mode_v[i];
        if (info) { info[0] = valid; info[1] = n_in; info[2] = steps; info[3] = rounds; }
    }
}

hipError_t launch_pose_sample(const PoseSampleArgs& a, const PoseSampleBufs& b, hipStream_t st) {
    for (int t = 1; t <= a.N; ++t) {
        hipLaunchKernelGGL(k_ps_samples, dim3((a.S + 63) / 64), dim3(64), 0, st, a, b, t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_ps_mode, dim3(1), dim3(kPsBlock), 0, st, a, b, t);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace vd
