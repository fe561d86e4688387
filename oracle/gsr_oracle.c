/*
 * gsr_oracle.c -- plain CPU reference ("oracle") for the tiled Gaussian
 * splatting RGB-D sensor renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the renderer library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * What it follows (paper: DISCOVERSE, arXiv 2507.21981):
 *   - Sec. III-A (Engine, "Renderer"): the renderer is the tile-based 3DGS
 *     rasteriser: sorting, splatting (projection of each 3D Gaussian to a 2D
 *     screen-space Gaussian), spherical-harmonics colour and alpha blending.
 *   - Sec. III-B ("Asset Formatting") and Fig. 1: a scene is a background
 *     node plus interactive nodes (objects, robots), each a Gaussian set
 *     placed by a rigid pose from the physics engine.
 *   - Sec. III-C (Sensor): RGB and depth frames come from alpha-compositing
 *     the colour and the camera-space z of the intersected Gaussians.
 *   - Sec. IV-B ("Mesh-Gaussian Transfer"): Gaussians are optimised with depth
 *     and opacity terms, which needs the gradient of the frames w.r.t. the
 *     Gaussian parameters (oracle analytic backward below).
 * The paper gives no equation for these steps; the definitions below are the
 * EWA-splatting model of the cited 3DGS renderer.  Readings where the paper
 * is silent (dilation 0.3 px^2, alpha clamp 0.99, skip below 1/255, stop when
 * transmittance would fall below 1e-4, pixel centres at +0.5, depth = sum of
 * alpha*T*z unnormalised, OpenCV camera axes, real SH with Condon-Shortley
 * phase and m = -l..l order) are listed with the design notes.
 *
 * Precision: every pixel, colour, projection and gradient value is FP64.
 * The candidate set and the blending order come from the FP32 "key
 * specification" path (or_keyspec), which states one exact FP32 operation
 * sequence (explicit fmaf, correctly rounded / and sqrt, no contraction; build
 * with -ffp-contract=off) for the tile rectangle and the depth key.  A GPU
 * implementation that follows the same sequence reproduces keys and tile
 * ranges bit for bit.
 *
 * Parity pins (tests/test_oracle_*.py): closed-form footprint of one
 * isotropic Gaussian, two-layer compositing, the 13-layer termination closed
 * form, brute force over all Gaussians without tiles, invariants (empty,
 * zero opacity, permutation, joint rigid motion), SH addition theorem and
 * quadrature orthonormality, Wigner-block orthogonality and composition, FP64
 * central finite differences of the analytic gradient.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXK 16

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics from the definition.                             */
/*                                                                           */
/* Y_l0 = N_l0 P_l(z),  Y_l,+m = sqrt2 N_lm P_l^m-part * Re((x+iy)^m),        */
/* Y_l,-m = sqrt2 N_lm P_l^m-part * Im((x+iy)^m), with                        */
/* N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and the Condon-Shortley phase     */
/* (-1)^m folded in: P_l^m(z) = (-1)^m (1-z^2)^(m/2) d^m P_l/dz^m, and on the */
/* unit sphere (1-z^2)^(m/2) {cos, sin}(m phi) = {Re, Im}((x+iy)^m).          */
/* These are polynomials in (x, y, z), differentiated symbolically below.    */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial coefficients, c[l][k] = coefficient of z^k in P_l,
   from Bonnet's recurrence (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}. */
static void legendre_coeffs(int L, double c[4][4]) {
    memset(c, 0, sizeof(double) * 16);
    c[0][0] = 1.0;
    if (L >= 1) c[1][1] = 1.0;
    for (int l = 1; l < L; ++l) {
        for (int k = 0; k <= l + 1; ++k) {
            double a = (k >= 1) ? (2.0 * l + 1.0) * c[l][k - 1] : 0.0;
            double b = (k <= l - 1) ? (double)l * c[l - 1][k] : 0.0;
            c[l + 1][k] = (a - b) / (l + 1.0);
        }
    }
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Evaluate Y_lm at the unit vector of `v` (v need not be unit length) and,
   if dY != NULL, the gradient of Y_lm(v/|v|) with respect to v:
   dY[idx*3 + j].  Index idx = l*l + (m + l). */
void or_sh_eval(int L, const double* v, double* Y, double* dY) {
    double c[4][4];
    legendre_coeffs(L, c);
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double x = v[0] / r, y = v[1] / r, z = v[2] / r;
    /* (x+iy)^m and its partials w.r.t. x and y. */
    double re[4], im[4], dre_dx[4], dim_dx[4], dre_dy[4], dim_dy[4];
    re[0] = 1.0; im[0] = 0.0;
    dre_dx[0] = dim_dx[0] = dre_dy[0] = dim_dy[0] = 0.0;
    for (int m = 1; m <= 3; ++m) {
        re[m] = re[m - 1] * x - im[m - 1] * y;
        im[m] = re[m - 1] * y + im[m - 1] * x;
        /* d/dx (x+iy)^m = m (x+iy)^(m-1); d/dy = i m (x+iy)^(m-1) */
        dre_dx[m] = m * re[m - 1];
        dim_dx[m] = m * im[m - 1];
        dre_dy[m] = -m * im[m - 1];
        dim_dy[m] = m * re[m - 1];
    }
    for (int l = 0; l <= L; ++l) {
        for (int m = 0; m <= l; ++m) {
            /* m-th derivative of P_l, evaluated at z, and its z-derivative. */
            double q = 0.0, dq = 0.0;
            for (int k = m; k <= l; ++k) {
                double coef = c[l][k];
                for (int t = 0; t < m; ++t) coef *= (double)(k - t);
                q += coef * pow(z, k - m);
                if (k - m >= 1) dq += coef * (k - m) * pow(z, k - m - 1);
            }
            double sign = (m % 2) ? -1.0 : 1.0;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            if (m == 0) {
                double k0 = N;
                int idx = l * l + l;
                Y[idx] = k0 * q;
                if (dY) { dY[idx * 3 + 0] = 0.0; dY[idx * 3 + 1] = 0.0; dY[idx * 3 + 2] = k0 * dq; }
            } else {
                double k0 = sign * sqrt(2.0) * N;
                int ip = l * l + l + m, in = l * l + l - m;
                Y[ip] = k0 * q * re[m];
                Y[in] = k0 * q * im[m];
                if (dY) {
                    dY[ip * 3 + 0] = k0 * q * dre_dx[m];
                    dY[ip * 3 + 1] = k0 * q * dre_dy[m];
                    dY[ip * 3 + 2] = k0 * dq * re[m];
                    dY[in * 3 + 0] = k0 * q * dim_dx[m];
                    dY[in * 3 + 1] = k0 * q * dim_dy[m];
                    dY[in * 3 + 2] = k0 * dq * im[m];
                }
            }
        }
    }
    if (dY) {
        /* chain through the normalisation u = v/|v|: du/dv = (I - u u^T)/|v| */
        int K = (L + 1) * (L + 1);
        double u[3] = {x, y, z};
        for (int i = 0; i < K; ++i) {
            double g[3] = {dY[i * 3 + 0], dY[i * 3 + 1], dY[i * 3 + 2]};
            double gu = g[0] * u[0] + g[1] * u[1] + g[2] * u[2];
            for (int j = 0; j < 3; ++j) dY[i * 3 + j] = (g[j] - gu * u[j]) / r;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Rotation of SH coefficients (pose application to a node's colour).        */
/* For each degree l the real SH span an invariant subspace, so             */
/* Y_l(R^T d) = D^l(R) Y_l(d) for a (2l+1)x(2l+1) matrix D^l.  The oracle    */
/* fits D^l by FP64 least squares on a fixed set of directions (any set of   */
/* >= 2l+1 generic directions determines it exactly).                       */
/* ------------------------------------------------------------------------ */
static int solve_spd(int n, double* A, double* B, int nrhs) {
    /* Gaussian elimination with partial pivoting: A X = B, A n x n, B n x nrhs (row-major). */
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (fabs(A[p * n + k]) < 1e-300) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
            for (int j = 0; j < nrhs; ++j) { double t = B[k * nrhs + j]; B[k * nrhs + j] = B[p * nrhs + j]; B[p * nrhs + j] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < nrhs; ++j) B[i * nrhs + j] -= f * B[k * nrhs + j];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < nrhs; ++j) {
            double s = B[k * nrhs + j];
            for (int i = k + 1; i < n; ++i) s -= A[k * n + i] * B[i * nrhs + j];
            B[k * nrhs + j] = s / A[k * n + k];
        }
    }
    return 0;
}

/* D[K*K] (row-major, block diagonal over degrees) with Y(R^T d) = D Y(d). */
int or_wigner(int L, const double* R, double* D) {
    int K = (L + 1) * (L + 1);
    memset(D, 0, sizeof(double) * K * K);
    enum { NS = 64 };
    double Ys[NS][OR_MAXK], Yr[NS][OR_MAXK];
    for (int s = 0; s < NS; ++s) {
        /* Fibonacci sphere directions */
        double zz = 1.0 - (2.0 * s + 1.0) / NS;
        double rr = sqrt(fmax(0.0, 1.0 - zz * zz));
        double ph = s * M_PI * (3.0 - sqrt(5.0));
        double d[3] = {rr * cos(ph), rr * sin(ph), zz};
        double dr[3];
        for (int i = 0; i < 3; ++i) dr[i] = R[0 * 3 + i] * d[0] + R[1 * 3 + i] * d[1] + R[2 * 3 + i] * d[2];
        or_sh_eval(L, d, Ys[s], NULL);
        or_sh_eval(L, dr, Yr[s], NULL);
    }
    for (int l = 0; l <= L; ++l) {
        int n = 2 * l + 1, o = l * l;
        double A[49], B[49];
        /* normal equations: (sum Y Y^T) D^T = sum Y Yr^T */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double a = 0.0, b = 0.0;
                for (int s = 0; s < NS; ++s) {
                    a += Ys[s][o + i] * Ys[s][o + j];
                    b += Ys[s][o + i] * Yr[s][o + j];
                }
                A[i * n + j] = a;
                B[i * n + j] = b;
            }
        if (solve_spd(n, A, B, n)) return -1;
        /* B now holds D^T */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) D[(o + i) * K + (o + j)] = B[j * n + i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Scene and camera description shared by the entry points.                  */
/* cam[] = { R00..R22 (world->camera, row-major), t0..t2, fx, fy, cx, cy,     */
/*           znear, bg0, bg1, bg2 }  (20 floats)                              */
/* pose_R[k*9], pose_t[k*3]: node-local -> world for node k.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, sh_degree;
    const double *means, *scales, *quats, *opac, *sh;
    const int32_t* node;
    int n_nodes;
    const double *pose_R, *pose_t;
} or_scene;

/* The FP32 key specification reads the original FP32 inputs. */
typedef struct {
    int n, sh_degree;
    const float *means, *scales, *quats, *opac;
    const int32_t* node;
    int n_nodes;
    const float *pose_R, *pose_t;
} or_scene32;

static void quat_rot64(const double* q, double* R) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[i * 3 + j] = A[i * 3 + 0] * B[0 * 3 + j] + A[i * 3 + 1] * B[1 * 3 + j] + A[i * 3 + 2] * B[2 * 3 + j];
}

/* ------------------------------------------------------------------------ */
/* FP32 key specification: tile rectangle, depth key and visibility.         */
/*                                                                           */
/* Per node k and camera c, the composed map camera<-node is formed in FP64   */
/* from the FP32 inputs, each sum evaluated left to right without fma, and   */
/* rounded once to FP32:                                                     */
/*   W_ij = (Rc_i0 Rk_0j + Rc_i1 Rk_1j) + Rc_i2 Rk_2j                         */
/*   w_i  = ((Rc_i0 tk_0 + Rc_i1 tk_1) + Rc_i2 tk_2) + tc_i                   */
/* Then per Gaussian, in FP32 with the operation order written below.        */
/* Visibility codes: 0 visible, 1 non-finite input, 2 opacity < 1/255,       */
/* 3 z <= znear, 4 zero quaternion, 5 det <= 0, 6 empty tile rectangle.      */
/* ------------------------------------------------------------------------ */
void or_compose_view(const float* cam, const float* pR, const float* pt, float* W, float* w) {
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double s = (double)cam[i * 3 + 0] * (double)pR[0 * 3 + j];
            s = s + (double)cam[i * 3 + 1] * (double)pR[1 * 3 + j];
            s = s + (double)cam[i * 3 + 2] * (double)pR[2 * 3 + j];
            W[i * 3 + j] = (float)s;
        }
        double s = (double)cam[i * 3 + 0] * (double)pt[0];
        s = s + (double)cam[i * 3 + 1] * (double)pt[1];
        s = s + (double)cam[i * 3 + 2] * (double)pt[2];
        s = s + (double)cam[9 + i];
        w[i] = (float)s;
    }
}

static int keyspec_one(const float* W, const float* w, const float* cam, int width, int height,
                       int tw, int th, const float* mu, const float* s, const float* q, float o,
                       int32_t* rect, uint32_t* zbits) {
    const float fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15], znear = cam[16];
    const int tiles_x = (width + tw - 1) / tw, tiles_y = (height + th - 1) / th;
    rect[0] = rect[1] = rect[2] = rect[3] = 0;
    *zbits = 0;
    for (int i = 0; i < 3; ++i)
        if (!isfinite(mu[i]) || !isfinite(s[i])) return 1;
    for (int i = 0; i < 4; ++i)
        if (!isfinite(q[i])) return 1;
    if (!isfinite(o)) return 1;
    if (!(o >= (float)(1.0 / 255.0))) return 2;
    float p[3];
    for (int r = 0; r < 3; ++r)
        p[r] = fmaf(W[r * 3 + 0], mu[0], fmaf(W[r * 3 + 1], mu[1], fmaf(W[r * 3 + 2], mu[2], w[r])));
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return 1;
    const float z = p[2];
    if (!(z > znear)) return 3;
    memcpy(zbits, &z, 4);
    const float iz = 1.0f / z;
    const float xz = p[0] * iz, yz = p[1] * iz;
    const float u = fmaf(fx, xz, cx), v = fmaf(fy, yz, cy);
    const float n2 = fmaf(q[0], q[0], fmaf(q[1], q[1], fmaf(q[2], q[2], q[3] * q[3])));
    if (!(n2 > 0.0f)) return 4;
    const float rn = 1.0f / sqrtf(n2);
    const float qw = q[0] * rn, qx = q[1] * rn, qy = q[2] * rn, qz = q[3] * rn;
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xzq = qx * qz, yzq = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    float R[9];
    R[0] = fmaf(-2.0f, yy + zz, 1.0f); R[1] = 2.0f * (xy - wz); R[2] = 2.0f * (xzq + wy);
    R[3] = 2.0f * (xy + wz); R[4] = fmaf(-2.0f, xx + zz, 1.0f); R[5] = 2.0f * (yzq - wx);
    R[6] = 2.0f * (xzq - wy); R[7] = 2.0f * (yzq + wx); R[8] = fmaf(-2.0f, xx + yy, 1.0f);
    float M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            float g = fmaf(W[r * 3 + 0], R[0 * 3 + c], fmaf(W[r * 3 + 1], R[1 * 3 + c], W[r * 3 + 2] * R[2 * 3 + c]));
            M[r * 3 + c] = g * s[c];
        }
    float S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            float v3 = fmaf(M[a * 3 + 0], M[b * 3 + 0], fmaf(M[a * 3 + 1], M[b * 3 + 1], M[a * 3 + 2] * M[b * 3 + 2]));
            S[a * 3 + b] = v3;
            S[b * 3 + a] = v3;
        }
    const float limx = 1.3f * ((0.5f * (float)width) / fx);
    const float limy = 1.3f * ((0.5f * (float)height) / fy);
    const float xc = fminf(fmaxf(xz, -limx), limx);
    const float yc = fminf(fmaxf(yz, -limy), limy);
    const float j00 = fx * iz, j11 = fy * iz;
    const float j02 = -(j00 * xc), j12 = -(j11 * yc);
    float T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
        T0[k] = fmaf(j00, S[0 * 3 + k], j02 * S[2 * 3 + k]);
        T1[k] = fmaf(j11, S[1 * 3 + k], j12 * S[2 * 3 + k]);
    }
    const float a = fmaf(T0[0], j00, T0[2] * j02) + 0.3f;
    const float b = fmaf(T0[1], j11, T0[2] * j12);
    const float c = fmaf(T1[1], j11, T1[2] * j12) + 0.3f;
    const float det = fmaf(a, c, -(b * b));
    if (!(det > 0.0f)) return 5;
    const float rx = fmaf(3.33f, sqrtf(a), 0.015625f);
    const float ry = fmaf(3.33f, sqrtf(c), 0.015625f);
    const float itw = 1.0f / (float)tw, ith = 1.0f / (float)th;
    const float xlo = (u - rx) * itw, xhi = (u + rx) * itw;
    const float ylo = (v - ry) * ith, yhi = (v + ry) * ith;
    const int tx0 = (int)fminf(fmaxf(floorf(xlo), 0.0f), (float)tiles_x);
    const int tx1 = (int)fminf(fmaxf(floorf(xhi) + 1.0f, 0.0f), (float)tiles_x);
    const int ty0 = (int)fminf(fmaxf(floorf(ylo), 0.0f), (float)tiles_y);
    const int ty1 = (int)fminf(fmaxf(floorf(yhi) + 1.0f, 0.0f), (float)tiles_y);
    if (tx0 >= tx1 || ty0 >= ty1) return 6;
    rect[0] = tx0; rect[1] = ty0; rect[2] = tx1; rect[3] = ty1;
    return 0;
}

/* Key-spec for every Gaussian of a scene seen by one camera.
   rect[n*4] = tx0, ty0, tx1, ty1 (exclusive), vis[n] (code), zbits[n] (the
   FP32 z bit pattern; set whenever z > znear was reached, i.e. codes 0, 4, 5
   and 6, zero otherwise). */
void or_keyspec(const or_scene32* sc, const float* cam, int width, int height, int tw, int th,
                int32_t* rect, uint32_t* zbits, int32_t* vis) {
    float* Wn = (float*)malloc(sizeof(float) * 12 * (size_t)(sc->n_nodes > 0 ? sc->n_nodes : 1));
    for (int k = 0; k < sc->n_nodes; ++k)
        or_compose_view(cam, sc->pose_R + 9 * k, sc->pose_t + 3 * k, Wn + 12 * k, Wn + 12 * k + 9);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < sc->n; ++i) {
        const int k = sc->node[i];
        vis[i] = keyspec_one(Wn + 12 * k, Wn + 12 * k + 9, cam, width, height, tw, th,
                             sc->means + 3 * (size_t)i, sc->scales + 3 * (size_t)i,
                             sc->quats + 4 * (size_t)i, sc->opac[i], rect + 4 * (size_t)i, zbits + i);
    }
    free(Wn);
}

/* ------------------------------------------------------------------------ */
/* FP64 projection ("splatting" + SH colour), Sec. III-A.                    */
/*                                                                           */
/* Pose (Fig. 1 / Sec. III-B): mu' = Rk mu + tk, rotation Rk R(q/|q|), SH    */
/* coefficients rotated per degree with the fitted D^l (k_world = D^T k).   */
/* Camera: p = Rc mu' + tc, z = p_z.  Sigma_w = (Rk R) diag(s)^2 (Rk R)^T.   */
/* EWA: J = [[fx/z, 0, -fx xc/z], [0, fy/z, -fy yc/z]] with xc = x/z, yc =   */
/* y/z clamped to +-1.3 * half-FoV tangent (the clamp enters J only);        */
/* Sigma2D = J Rc Sigma_w Rc^T J^T + 0.3 I; conic Q = Sigma2D^-1;            */
/* u = fx x/z + cx, v = fy y/z + cy.  Colour c = max(0, sum k Y(d) + 0.5)    */
/* with d the unit vector from the camera centre to mu'.                     */
/* geo[i*28]: u v A B C o r g b z, a b c (Sigma2D), then the FP32 error-bound  */
/* quantities of fp32_bounds (13..24), rest unused.                          */
/* ------------------------------------------------------------------------ */
#define GEO 28

typedef struct {
    double Rk[9], tk[3], D[OR_MAXK * OR_MAXK];
} node64;

static void prep_nodes(const or_scene* sc, node64* nd) {
    for (int k = 0; k < sc->n_nodes; ++k) {
        for (int i = 0; i < 9; ++i) nd[k].Rk[i] = sc->pose_R[9 * k + i];
        for (int i = 0; i < 3; ++i) nd[k].tk[i] = sc->pose_t[3 * k + i];
        or_wigner(sc->sh_degree, nd[k].Rk, nd[k].D);
    }
}

typedef struct {
    double Rc[9], tc[3], fx, fy, cx, cy, limx, limy, centre[3];
} cam64;

static void prep_cam(const double* cam, int width, int height, cam64* c) {
    for (int i = 0; i < 9; ++i) c->Rc[i] = cam[i];
    for (int i = 0; i < 3; ++i) c->tc[i] = cam[9 + i];
    c->fx = cam[12]; c->fy = cam[13]; c->cx = cam[14]; c->cy = cam[15];
    c->limx = 1.3 * (0.5 * width / c->fx);
    c->limy = 1.3 * (0.5 * height / c->fy);
    for (int i = 0; i < 3; ++i)
        c->centre[i] = -(c->Rc[0 * 3 + i] * c->tc[0] + c->Rc[1 * 3 + i] * c->tc[1] + c->Rc[2 * 3 + i] * c->tc[2]);
}

/* Everything the backward needs about one Gaussian in one camera, and the FP32 error
   bounds of its screen-space quantities (see fp32_bounds). */
typedef struct {
    double mu_w[3], Rg[9], s[3], p[3], Sc[9], J[6], S2[3], Q[3], u, v, o, col[3], colpre[3];
    double dvec[3], kw[OR_MAXK * 3];
    double eu, ev, edet, dj, ajx, ajy, smax, ssum;
    int clampx, clampy;
} proj64;

/* ------------------------------------------------------------------------ */
/* FP32 error bounds of the screen-space quantities.                         */
/*                                                                           */
/* An FP32 renderer computes u, v and the dilated 2D covariance from FP32    */
/* inputs with the key-specification operations (camera<-node map rounded    */
/* once to FP32, fma chains, correctly rounded division and square root).    */
/* With U = 2^-24 the unit roundoff and each operation contributing at most  */
/* U times the sum of the magnitudes of its terms, to first order:           */
/*   p_r = W_r . mu + w_r          |dp_r| <= 4U a_r,  a_r = sum_j |W_rj mu_j| + |w_r| */
/*   x/z                           |d(x/z)| <= |x/z| (2U + dz/z) + dp_0/z    */
/*   u = fx x/z + cx               eu = fx |d(x/z)| + U |u|   (same for v)   */
/*   J entries                     relative error dj = 3U + dz/z, and j02 also */
/*                                 moves by j00 |d(x/z)| (fx dxc below), j12 likewise */
/*   M = (W R(q)) diag(s)          M + E diag(s) with |E_rc| <= 18U (rotation from */
/*                                 the normalised quaternion, W rounded, 3-term sums) */
/*   Sigma = M M^T                 3-term dot products, error <= 3U sum_c |M_ac M_bc| */
/*   Sigma2D = J Sigma J^T + 0.3 I two more 2-term fma levels: 4U |J||Sigma||J|^T */
/*   det = a c - b^2, conic = adj / det   relative edet = U (b^2 + det) / det + 4U */
/* The exponent depends on the covariance through the quadratic form          */
/* g^T Sigma2D g with g = Q d (decision_bound), so the bound is taken on that */
/* form directly: with y = J^T g, y' = |J|^T |g| and q = y^T Sigma y,        */
/*   |g^T dSigma2D g| <= 108U s_max |y| sqrt(q) + (54U s_max |y|)^2          */
/*                       + 3U (sum s^2) |y|^2 + 2 s_max |dJ^T g| sqrt(q)     */
/*                       + 4U (sum s^2) |y'|^2 + 2U 0.3 |g|^2                */
/* (errors of M enter linearly in s_max, roundings of entries of size s_max^2 */
/* quadratically, which is how the form of a thin splat loses accuracy).     */
/* geo[13..24] keep eu, ev, edet, j00, j11, j02, j12, dj, fx dxc, fy dyc,     */
/* s_max, sum s^2.                                                            */
/* ------------------------------------------------------------------------ */
#define OR_U 5.9604644775390625e-08

static void fp32_bounds(const node64* N, const cam64* c, const double* mu, proj64* P) {
    const double U = OR_U;
    double W[9], w[3], a[3];
    matmul3(c->Rc, N->Rk, W);
    for (int r = 0; r < 3; ++r) {
        w[r] = c->Rc[r * 3 + 0] * N->tk[0] + c->Rc[r * 3 + 1] * N->tk[1] + c->Rc[r * 3 + 2] * N->tk[2] + c->tc[r];
        a[r] = fabs(W[r * 3 + 0] * mu[0]) + fabs(W[r * 3 + 1] * mu[1]) + fabs(W[r * 3 + 2] * mu[2]) + fabs(w[r]);
    }
    const double z = P->p[2], dz = 4.0 * U * a[2];
    const double xz = P->p[0] / z, yz = P->p[1] / z;
    const double dxz = fabs(xz) * (2.0 * U + dz / z) + 4.0 * U * a[0] / z;
    const double dyz = fabs(yz) * (2.0 * U + dz / z) + 4.0 * U * a[1] / z;
    P->eu = c->fx * dxz + U * fabs(P->u);
    P->ev = c->fy * dyz + U * fabs(P->v);
    /* beyond the clamp the FP32 limit (1.3f (0.5 W / fx)) moves by a few U */
    const double dxc = P->clampx ? 4.0 * U * c->limx : dxz;
    const double dyc = P->clampy ? 4.0 * U * c->limy : dyz;
    P->dj = 3.0 * U + dz / z;
    P->ajx = c->fx / z * dxc;
    P->ajy = c->fy / z * dyc;
    P->smax = fmax(P->s[0], fmax(P->s[1], P->s[2]));
    P->ssum = P->s[0] * P->s[0] + P->s[1] * P->s[1] + P->s[2] * P->s[2];
    const double det = P->S2[0] * P->S2[2] - P->S2[1] * P->S2[1];
    P->edet = U * (P->S2[1] * P->S2[1] + fabs(det)) / det + 4.0 * U;
}

static void project64(const or_scene* sc, const node64* nd, const cam64* c, int i, proj64* P) {
    const int k = sc->node[i];
    const int L = sc->sh_degree, K = (L + 1) * (L + 1);
    const node64* N = nd + k;
    double mu[3], q[4], Rq[9];
    for (int j = 0; j < 3; ++j) { mu[j] = sc->means[3 * (size_t)i + j]; P->s[j] = sc->scales[3 * (size_t)i + j]; }
    for (int j = 0; j < 4; ++j) q[j] = sc->quats[4 * (size_t)i + j];
    P->o = sc->opac[i];
    for (int r = 0; r < 3; ++r)
        P->mu_w[r] = N->Rk[r * 3 + 0] * mu[0] + N->Rk[r * 3 + 1] * mu[1] + N->Rk[r * 3 + 2] * mu[2] + N->tk[r];
    quat_rot64(q, Rq);
    matmul3(N->Rk, Rq, P->Rg);
    for (int r = 0; r < 3; ++r)
        P->p[r] = c->Rc[r * 3 + 0] * P->mu_w[0] + c->Rc[r * 3 + 1] * P->mu_w[1] + c->Rc[r * 3 + 2] * P->mu_w[2] + c->tc[r];
    /* Sigma_w = Rg diag(s^2) Rg^T, then Sigma_c = Rc Sigma_w Rc^T */
    double Sw[9], A[9], Sc[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0;
            for (int j = 0; j < 3; ++j) t += P->Rg[a * 3 + j] * P->s[j] * P->s[j] * P->Rg[b * 3 + j];
            Sw[a * 3 + b] = t;
        }
    matmul3(c->Rc, Sw, A);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Sc[a * 3 + b] = A[a * 3 + 0] * c->Rc[b * 3 + 0] + A[a * 3 + 1] * c->Rc[b * 3 + 1] + A[a * 3 + 2] * c->Rc[b * 3 + 2];
    memcpy(P->Sc, Sc, sizeof(Sc));
    const double x = P->p[0], y = P->p[1], z = P->p[2];
    double xz = x / z, yz = y / z;
    P->clampx = (xz < -c->limx || xz > c->limx);
    P->clampy = (yz < -c->limy || yz > c->limy);
    double xcl = fmin(fmax(xz, -c->limx), c->limx), ycl = fmin(fmax(yz, -c->limy), c->limy);
    double *J = P->J;
    J[0] = c->fx / z; J[1] = 0.0; J[2] = -c->fx * xcl / z;
    J[3] = 0.0; J[4] = c->fy / z; J[5] = -c->fy * ycl / z;
    /* Sigma2D = J Sc J^T + 0.3 I */
    double JS[6];
    for (int r = 0; r < 2; ++r)
        for (int j = 0; j < 3; ++j) JS[r * 3 + j] = J[r * 3 + 0] * Sc[0 * 3 + j] + J[r * 3 + 1] * Sc[1 * 3 + j] + J[r * 3 + 2] * Sc[2 * 3 + j];
    double a2 = JS[0] * J[0] + JS[1] * J[1] + JS[2] * J[2] + 0.3;
    double b2 = JS[0] * J[3] + JS[1] * J[4] + JS[2] * J[5];
    double c2 = JS[3] * J[3] + JS[4] * J[4] + JS[5] * J[5] + 0.3;
    P->S2[0] = a2; P->S2[1] = b2; P->S2[2] = c2;
    double det = a2 * c2 - b2 * b2;
    P->Q[0] = c2 / det; P->Q[1] = -b2 / det; P->Q[2] = a2 / det;
    P->u = c->fx * x / z + c->cx;
    P->v = c->fy * y / z + c->cy;
    /* colour: world-frame coefficients k_w = D^T k */
    double dv[3] = {P->mu_w[0] - c->centre[0], P->mu_w[1] - c->centre[1], P->mu_w[2] - c->centre[2]};
    memcpy(P->dvec, dv, sizeof(dv));
    double Y[OR_MAXK];
    or_sh_eval(L, dv, Y, NULL);
    const double* shi = sc->sh + (size_t)i * K * 3;
    for (int ch = 0; ch < 3; ++ch) {
        for (int m = 0; m < K; ++m) {
            double t = 0;
            for (int j = 0; j < K; ++j) t += N->D[j * K + m] * shi[j * 3 + ch];
            P->kw[m * 3 + ch] = t;
        }
        double sum = 0;
        for (int m = 0; m < K; ++m) sum += P->kw[m * 3 + ch] * Y[m];
        P->colpre[ch] = sum + 0.5;
        P->col[ch] = fmax(0.0, sum + 0.5);
    }
    fp32_bounds(N, c, mu, P);
}

/* FP64 projection of every Gaussian (geo[i*GEO]) for one camera. */
void or_project(const or_scene* sc, const double* cam, int width, int height, double* geo) {
    node64* nd = (node64*)malloc(sizeof(node64) * (size_t)(sc->n_nodes > 0 ? sc->n_nodes : 1));
    prep_nodes(sc, nd);
    cam64 c;
    prep_cam(cam, width, height, &c);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < sc->n; ++i) {
        proj64 P;
        double* g = geo + (size_t)i * GEO;
        memset(g, 0, sizeof(double) * GEO);
        project64(sc, nd, &c, i, &P);
        g[0] = P.u; g[1] = P.v; g[2] = P.Q[0]; g[3] = P.Q[1]; g[4] = P.Q[2]; g[5] = P.o;
        g[6] = P.col[0]; g[7] = P.col[1]; g[8] = P.col[2]; g[9] = P.p[2];
        g[10] = P.S2[0]; g[11] = P.S2[1]; g[12] = P.S2[2];
        g[13] = P.eu; g[14] = P.ev; g[15] = P.edet; g[16] = P.J[0]; g[17] = P.J[4]; g[18] = P.J[2];
        g[19] = P.J[5]; g[20] = P.dj; g[21] = P.ajx; g[22] = P.ajy; g[23] = P.smax; g[24] = P.ssum;
    }
    free(nd);
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing (alpha blending, Sec. III-A; RGB and depth,         */
/* Sec. III-C), front to back in key order:                                 */
/*   power = -1/2 (A dx^2 + C dy^2) - B dx dy, dx = px + 0.5 - u, ...;       */
/*   skip if power > 0; alpha = min(0.99, o exp(power)); skip if alpha <     */
/*   1/255; if T (1 - alpha) < 1e-4 stop without blending this entry;       */
/*   else C += alpha T c, D += alpha T z, T *= (1 - alpha).                  */
/* Outputs rgb = C + T bg, depth = D, alpha = 1 - T.                         */
/*                                                                           */
/* Ambiguous decisions.  Near a threshold an FP32 renderer can take the     */
/* other branch, and both results are correct.  decision_bound gives, from  */
/* the FP32 bounds of u, v and Sigma2D (fp32_bounds), a bound on the        */
/* error of an FP32 alpha in log units (|d ln alpha| = |d power|):          */
/*   |d power| <= |g_x| du' + |g_y| dv' + 1/2 g^T eS g + 1/2 m edet          */
/*                + 6U (m_abs / 2 + |ln o|) + 4U                             */
/* with g = Q d (the exponent's gradient in u, v), m = d^T Q d, du' = eu +   */
/* U |dx| (the subtraction), m_abs the form with absolute values, the 6U    */
/* term the evaluation of the exponent in FP32 and the 4U term exp and log.  */
/* The transmittance test T (1 - alpha) carries the log errors of the       */
/* alphas blended before it, each amplified by alpha / (1 - alpha), plus two */
/* roundings per blend.  Those come from the roundings of different         */
/* Gaussians' projections and of separate products, which are independent,  */
/* so they are accumulated as a root sum of squares (the square-root growth */
/* of independent rounding errors, Higham, Accuracy and Stability of        */
/* Numerical Algorithms, sec. 2.8) of the per-blend worst cases, rather than */
/* by their sum, which would grow with the number of layers and mark a      */
/* large share of the stopping decisions of deep pixels as ambiguous.       */
/* A decision whose log-distance to its threshold                           */
/* (|ln alpha - ln(1/255)|, |ln(T (1 - alpha)) - ln 1e-4|) is below         */
/* safety x bound + floor is ambiguous; the pixel is                         */
/* reported with the result of its most ambiguous decision (smallest        */
/* distance / bound) flipped as an equally valid alternative; a pixel with  */
/* two or more ambiguous decisions is flagged (out_flags bit 1).            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rgb[3], depth, T;
    int last, evals;
    int64_t trace;
    double min_margin;
    int amb_count, amb_j, amb_type;
} pixres;

/* bound of |ln alpha_FP32 - ln alpha| for alpha = o exp(power) at offset (dx, dy) */
static double decision_bound(const double* g, double dx, double dy) {
    const double U = OR_U;
    const double A = g[2], B = g[3], C = g[4];
    const double gx = A * dx + B * dy, gy = B * dx + C * dy;
    const double m = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy;
    const double m_abs = fabs(A) * dx * dx + 2.0 * fabs(B * dx * dy) + fabs(C) * dy * dy;
    const double du = g[13] + U * fabs(dx), dv = g[14] + U * fabs(dy);
    /* the quadratic form g^T dSigma2D g (fp32_bounds) */
    const double j00 = g[16], j11 = g[17], j02 = g[18], j12 = g[19];
    const double y0 = j00 * gx, y1 = j11 * gy, y2 = j02 * gx + j12 * gy;
    const double ny = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    const double a0 = j00 * fabs(gx), a1 = j11 * fabs(gy), a2 = fabs(j02 * gx) + fabs(j12 * gy);
    const double na2 = a0 * a0 + a1 * a1 + a2 * a2;
    const double q = fmax(0.0, (g[10] - 0.3) * gx * gx + 2.0 * g[11] * gx * gy + (g[12] - 0.3) * gy * gy);
    const double smax = g[23], ssum = g[24];
    const double dJg = g[20] * sqrt(na2) + g[21] * fabs(gx) + g[22] * fabs(gy);
    const double form = 108.0 * U * smax * ny * sqrt(q) + (54.0 * U * smax * ny) * (54.0 * U * smax * ny) +
                        3.0 * U * ssum * ny * ny + 2.0 * smax * dJg * sqrt(q) + 4.0 * U * ssum * na2 +
                        0.6 * U * (gx * gx + gy * gy);
    return fabs(gx) * du + fabs(gy) * dv + 0.5 * form + 0.5 * fabs(m) * g[15] +
           6.0 * U * (0.5 * m_abs + fabs(log(g[5]))) + 4.0 * U;
}

static void composite_pixel(const int32_t* list, int64_t cnt, const double* geo, const double* bg,
                            double px, double py, int flip_j, int flip_type,
                            double safety, double floor_, pixres* R) {
    const double U = OR_U;
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
    double eT2 = 0.0; /* sum of squares of the blends' contributions to the log error of T */
    int last = 0, evals = 0;
    int64_t trace = 0;
    R->min_margin = INFINITY;
    R->amb_count = 0; R->amb_j = -1; R->amb_type = -1;
    const double athr = 1.0 / 255.0;
    for (int64_t j = 0; j < cnt; ++j) {
        const double* g = geo + (size_t)list[j] * GEO;
        ++evals;
        double dx = px - g[0], dy = py - g[1];
        double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
        if (power > 0.0) continue;
        double oG = g[5] * exp(power);
        double alpha = fmin(0.99, oG);
        const double ea = decision_bound(g, dx, dy);
        /* log-distance to the threshold over the bound: below 1 the decision is ambiguous */
        double ra = fabs(log(alpha / athr)) / (safety * ea + floor_);
        int skip = alpha < athr;
        if (ra < 1.0) { R->amb_count++; if (ra < R->min_margin) { R->min_margin = ra; R->amb_j = (int)j; R->amb_type = 0; } }
        else if (ra < R->min_margin) R->min_margin = ra;
        if (flip_j == (int)j && flip_type == 0) skip = !skip;
        if (skip) continue;
        /* an FP32 alpha equals the FP32 clamp value when both sides surely clamp */
        const double ea_eff = (oG * (1.0 - ea) >= 0.99 ? 0.0 : ea) + 1e-8;
        const double cT = (ea_eff + U) * alpha / (1.0 - alpha) + U;
        const double eTn = sqrt(eT2 + cT * cT);
        double test = T * (1.0 - alpha);
        double rt = fabs(log(test / 1e-4)) / (safety * eTn + floor_);
        int stop = test < 1e-4;
        if (rt < 1.0) { R->amb_count++; if (rt < R->min_margin) { R->min_margin = rt; R->amb_j = (int)j; R->amb_type = 1; } }
        else if (rt < R->min_margin) R->min_margin = rt;
        if (flip_j == (int)j && flip_type == 1) stop = !stop;
        if (stop) break;
        double wgt = alpha * T;
        C[0] += wgt * g[6]; C[1] += wgt * g[7]; C[2] += wgt * g[8];
        D += wgt * g[9];
        T = test;
        eT2 += cT * cT;
        last = (int)j + 1;
        /* decision trace: which entries were blended, and whether the 0.99 clamp was active */
        trace += (int64_t)(j + 1) * (oG >= 0.99 ? 1000003 : 1);
    }
    R->trace = trace + evals;
    for (int ch = 0; ch < 3; ++ch) R->rgb[ch] = C[ch] + T * bg[ch];
    R->depth = D;
    R->T = T;
    R->last = last;
    R->evals = evals;
}

/* Composite an image from per-tile sorted candidate lists.
   ranges[t*2] = [start, end) into vals (indices into geo).
   Per pixel out: rgb[3] depth alpha, Tfin, last (entries up to the last blended one),
   evals, margin (smallest ratio of a decision's distance to its threshold over its FP32
   bound; below 1 the decision is ambiguous), flags (bit0: ambiguous, alternative provided;
   bit1: >= 2 ambiguous decisions, bit2: the most ambiguous one is a stopping decision),
   alt[5] = rgb depth alpha of the flipped branch, trace = a checksum of
   the discrete decisions (which entries were blended, clamp states). */
void or_composite(int width, int height, int tw, int th, const int64_t* ranges, const int32_t* vals,
                  const double* geo, const float* bgf, double safety, double floor_,
                  double* rgb, double* depth, double* alpha, double* Tfin, int32_t* last,
                  int32_t* evals, double* margin, int32_t* flags, double* alt, int64_t* trace) {
    const int tiles_x = (width + tw - 1) / tw;
    const double bg[3] = {bgf[0], bgf[1], bgf[2]};
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < height; ++py) {
        for (int px = 0; px < width; ++px) {
            const int t = (py / th) * tiles_x + (px / tw);
            const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
            pixres R;
            composite_pixel(vals + s, e - s, geo, bg, px + 0.5, py + 0.5, -1, -1, safety, floor_, &R);
            const size_t p = (size_t)py * width + px;
            rgb[3 * p + 0] = R.rgb[0]; rgb[3 * p + 1] = R.rgb[1]; rgb[3 * p + 2] = R.rgb[2];
            depth[p] = R.depth; alpha[p] = 1.0 - R.T; Tfin[p] = R.T; last[p] = R.last; evals[p] = R.evals;
            trace[p] = R.trace;
            margin[p] = R.min_margin;
            int fl = 0;
            double* a = alt + 5 * p;
            a[0] = R.rgb[0]; a[1] = R.rgb[1]; a[2] = R.rgb[2]; a[3] = R.depth; a[4] = 1.0 - R.T;
            if (R.amb_count >= 1) {
                pixres F;
                composite_pixel(vals + s, e - s, geo, bg, px + 0.5, py + 0.5, R.amb_j, R.amb_type, safety, floor_, &F);
                a[0] = F.rgb[0]; a[1] = F.rgb[1]; a[2] = F.rgb[2]; a[3] = F.depth; a[4] = 1.0 - F.T;
                fl |= 1;
                if (R.amb_count >= 2) fl |= 2;
                if (R.amb_type == 1) fl |= 4;
            }
            flags[p] = fl;
        }
    }
}

/* The same per-pixel definition at a list of pixels (pix[i] = py * width + px); out[i*8] =
   r g b depth alpha T last evals, flags[i], alt[i*5]. */
void or_composite_sample(int width, int height, int tw, int th, const int64_t* ranges, const int32_t* vals,
                         const double* geo, const float* bgf, double safety, double floor_,
                         const int64_t* pix, int64_t npix, double* out, int32_t* flags, double* alt) {
    const int tiles_x = (width + tw - 1) / tw;
    const double bg[3] = {bgf[0], bgf[1], bgf[2]};
    (void)height;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < npix; ++i) {
        const int px = (int)(pix[i] % width), py = (int)(pix[i] / width);
        const int t = (py / th) * tiles_x + (px / tw);
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        pixres R;
        composite_pixel(vals + s, e - s, geo, bg, px + 0.5, py + 0.5, -1, -1, safety, floor_, &R);
        double* o = out + 8 * i;
        o[0] = R.rgb[0]; o[1] = R.rgb[1]; o[2] = R.rgb[2]; o[3] = R.depth; o[4] = 1.0 - R.T; o[5] = R.T;
        o[6] = R.last; o[7] = R.evals;
        double* a = alt + 5 * i;
        a[0] = R.rgb[0]; a[1] = R.rgb[1]; a[2] = R.rgb[2]; a[3] = R.depth; a[4] = 1.0 - R.T;
        int fl = 0;
        if (R.amb_count >= 1) {
            pixres F;
            composite_pixel(vals + s, e - s, geo, bg, px + 0.5, py + 0.5, R.amb_j, R.amb_type, safety, floor_, &F);
            a[0] = F.rgb[0]; a[1] = F.rgb[1]; a[2] = F.rgb[2]; a[3] = F.depth; a[4] = 1.0 - F.T;
            fl |= 1;
            if (R.amb_count >= 2) fl |= 2;
            if (R.amb_type == 1) fl |= 4;
        }
        flags[i] = fl;
    }
}

/* ------------------------------------------------------------------------ */
/* Analytic backward, FP64.                                                  */
/*                                                                           */
/* Stage 1 (per pixel, compositing): for each blended entry i, with          */
/* T_i the transmittance in front of it, S^C_i = sum_{j>i} c_j a_j T_j +     */
/* T_f bg and S^D_i = sum_{j>i} z_j a_j T_j:                                 */
/*   dL/dc_i += gC a_i T_i,  dL/dz_i += gD a_i T_i,                          */
/*   dL/da_i  = gC.(c_i T_i - S^C_i/(1-a_i)) + gD (z_i T_i - S^D_i/(1-a_i))  */
/*              + gA T_f/(1-a_i);                                            */
/* through a = o G (zero where the 0.99 clamp is active) and G = exp(power)  */
/* to o, u, v and the conic.                                                 */
/* g2d[i*10]: du dv dA dB dC do dr dg db dz                                   */
/* ------------------------------------------------------------------------ */
#define G2D 10

/* Backward of one pixel's compositing: recompute the forward walk, then accumulate the 2D
   gradients of its blended entries back to front (serial: fixed accumulation order). */
typedef struct {
    int cap;
    int* ent;
    double *ea, *eT;
} bwd_scratch;

static void backward_pixel(const int32_t* list, int64_t cnt, const double* geo, const double* bg, int px, int py,
                           const double* gC, double gD, double gA, double* g2d, bwd_scratch* w) {
    const double fx = px + 0.5, fy = py + 0.5;
    double T = 1.0;
    int nb = 0;
    for (int64_t j = 0; j < cnt; ++j) {
        const double* g = geo + (size_t)list[j] * GEO;
        double dx = fx - g[0], dy = fy - g[1];
        double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
        if (power > 0.0) continue;
        double alpha = fmin(0.99, g[5] * exp(power));
        if (alpha < 1.0 / 255.0) continue;
        double test = T * (1.0 - alpha);
        if (test < 1e-4) break;
        if (nb == w->cap) {
            w->cap *= 2;
            w->ent = (int*)realloc(w->ent, sizeof(int) * w->cap);
            w->ea = (double*)realloc(w->ea, sizeof(double) * w->cap);
            w->eT = (double*)realloc(w->eT, sizeof(double) * w->cap);
        }
        w->ent[nb] = list[j]; w->ea[nb] = alpha; w->eT[nb] = T; ++nb;
        T = test;
    }
    const double Tf = T;
    double SC[3] = {Tf * bg[0], Tf * bg[1], Tf * bg[2]}, SD = 0.0;
    for (int k = nb - 1; k >= 0; --k) {
        const int i = w->ent[k];
        const double* g = geo + (size_t)i * GEO;
        double* o = g2d + (size_t)i * G2D;
        const double a = w->ea[k], Ti = w->eT[k], wt = a * Ti;
        o[6] += gC[0] * wt; o[7] += gC[1] * wt; o[8] += gC[2] * wt;
        o[9] += gD * wt;
        double dLda = 0.0;
        for (int ch = 0; ch < 3; ++ch) dLda += gC[ch] * (g[6 + ch] * Ti - SC[ch] / (1.0 - a));
        dLda += gD * (g[9] * Ti - SD / (1.0 - a));
        dLda += gA * Tf / (1.0 - a);
        for (int ch = 0; ch < 3; ++ch) SC[ch] += g[6 + ch] * wt;
        SD += g[9] * wt;
        double dx = fx - g[0], dy = fy - g[1];
        double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
        double G = exp(power);
        if (g[5] * G < 0.99) {
            o[5] += dLda * G;
            double dp = dLda * g[5] * G;
            o[0] += dp * (g[2] * dx + g[3] * dy);
            o[1] += dp * (g[4] * dy + g[3] * dx);
            o[2] += dp * (-0.5 * dx * dx);
            o[3] += dp * (-dx * dy);
            o[4] += dp * (-0.5 * dy * dy);
        }
    }
}

void or_backward_2d(int width, int height, int tw, int th, const int64_t* ranges, const int32_t* vals,
                    const double* geo, const float* bgf, const double* g_rgb, const double* g_depth,
                    const double* g_alpha, int n, double* g2d) {
    const int tiles_x = (width + tw - 1) / tw;
    const double bg[3] = {bgf[0], bgf[1], bgf[2]};
    memset(g2d, 0, sizeof(double) * G2D * (size_t)n);
    bwd_scratch w = {1024, (int*)malloc(sizeof(int) * 1024), (double*)malloc(sizeof(double) * 1024),
                     (double*)malloc(sizeof(double) * 1024)};
    for (int py = 0; py < height; ++py) {
        for (int px = 0; px < width; ++px) {
            const int t = (py / th) * tiles_x + (px / tw);
            const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
            const size_t p = (size_t)py * width + px;
            const double gC[3] = {g_rgb[3 * p], g_rgb[3 * p + 1], g_rgb[3 * p + 2]};
            backward_pixel(vals + s, e - s, geo, bg, px, py, gC, g_depth ? g_depth[p] : 0.0,
                           g_alpha ? g_alpha[p] : 0.0, g2d, &w);
        }
    }
    free(w.ent); free(w.ea); free(w.eT);
}

/* The same at a list of pixels (pix[i] = py * width + px) with upstream gradients g_rgb[3i],
   g_depth[i], g_alpha[i] (either of the last two may be NULL); every other pixel has zero
   upstream gradient and contributes nothing. */
void or_backward_2d_sample(int width, int height, int tw, int th, const int64_t* ranges, const int32_t* vals,
                           const double* geo, const float* bgf, const int64_t* pix, int64_t npix,
                           const double* g_rgb, const double* g_depth, const double* g_alpha, int n, double* g2d) {
    const int tiles_x = (width + tw - 1) / tw;
    const double bg[3] = {bgf[0], bgf[1], bgf[2]};
    (void)height;
    memset(g2d, 0, sizeof(double) * G2D * (size_t)n);
    bwd_scratch w = {1024, (int*)malloc(sizeof(int) * 1024), (double*)malloc(sizeof(double) * 1024),
                     (double*)malloc(sizeof(double) * 1024)};
    for (int64_t i = 0; i < npix; ++i) {
        const int px = (int)(pix[i] % width), py = (int)(pix[i] / width);
        const int t = (py / th) * tiles_x + (px / tw);
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        backward_pixel(vals + s, e - s, geo, bg, px, py, g_rgb + 3 * i, g_depth ? g_depth[i] : 0.0,
                       g_alpha ? g_alpha[i] : 0.0, g2d, &w);
    }
    free(w.ent); free(w.ea); free(w.eT);
}

/* Stage 2 (per Gaussian, projection): chain the 2D gradients to the node-   */
/* local parameters.  Conic Q = Sigma2D^-1 gives dL/dSigma2D = -Q G Q with   */
/* G = [[dA, dB/2], [dB/2, dC]]; Sigma2D = J Sc J^T gives dSc = J^T H J and  */
/* dJ = 2 H J Sc; u, v, J and z depend on p = Rc mu' + tc; Sc = Rc Sw Rc^T;  */
/* Sw = M M^T with M = Rg diag(s), Rg = Rk R(q/|q|); colour through the SH   */
/* basis and the view direction; mu' = Rk mu + tk; k_w = D^T k.              */
/* Outputs are ACCUMULATED into the gradient arrays (same layout as inputs). */
/* Node poses (Sec. III-B: each node is placed by a rigid pose from the physics engine).      */
/* With d_pose != NULL the gradient with respect to each node's pose is ACCUMULATED into     */
/* d_pose[k*6] = (omega, rho): the derivative along the world-frame left perturbation        */
/* R' = exp([omega]x) R_k, t' = exp([omega]x) t_k + rho.  To first order it moves each of    */
/* the node's world means by omega x mu' + rho and each world rotation frame Rg by          */
/* [omega]x Rg, and (colour = k_w . Y(d), k_w = D(R')^T k, with D(e^[omega] R) =            */
/* D(R) D(e^[omega])) turns the colour's view vector mu' - c into mu' - c + rho + omega x c,  */
/* so with g_mu the gradient of the world mean through the projection, g_v that of the      */
/* view vector through the colour and G that of Rg:                                         */
/*   d rho   = sum_i g_mu + g_v                                                             */
/*   d omega = sum_i mu' x g_mu + c x g_v + (M_21 - M_12, M_02 - M_20, M_10 - M_01),       */
/*             M = G Rg^T.                                                                   */
void or_backward_project(const or_scene* sc, const double* cam, int width, int height, const double* g2d,
                         double* d_means, double* d_scales, double* d_quats, double* d_opac, double* d_sh,
                         double* d_pose) {
    node64* nd = (node64*)malloc(sizeof(node64) * (size_t)(sc->n_nodes > 0 ? sc->n_nodes : 1));
    prep_nodes(sc, nd);
    cam64 c;
    prep_cam(cam, width, height, &c);
    const int L = sc->sh_degree, K = (L + 1) * (L + 1);
    /* per-Gaussian pose contributions, summed per node in a fixed order after the loop */
    double* pg = d_pose ? (double*)calloc((size_t)(sc->n > 0 ? sc->n : 1) * 6, sizeof(double)) : NULL;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < sc->n; ++i) {
        const double* gg = g2d + (size_t)i * G2D;
        int any = 0;
        for (int j = 0; j < G2D; ++j) any |= (gg[j] != 0.0);
        if (!any) continue;
        proj64 P;
        project64(sc, nd, &c, i, &P);
        const node64* N = nd + sc->node[i];
        const double x = P.p[0], y = P.p[1], z = P.p[2];
        double dp[3] = {0, 0, 0};
        /* u, v */
        dp[0] += gg[0] * c.fx / z;
        dp[2] += gg[0] * (-c.fx * x / (z * z));
        dp[1] += gg[1] * c.fy / z;
        dp[2] += gg[1] * (-c.fy * y / (z * z));
        /* depth z */
        dp[2] += gg[9];
        /* conic -> Sigma2D */
        double Qm[4] = {P.Q[0], P.Q[1], P.Q[1], P.Q[2]};
        double Gm[4] = {gg[2], 0.5 * gg[3], 0.5 * gg[3], gg[4]};
        double QG[4], H[4];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) QG[a * 2 + b] = Qm[a * 2 + 0] * Gm[0 * 2 + b] + Qm[a * 2 + 1] * Gm[1 * 2 + b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) H[a * 2 + b] = -(QG[a * 2 + 0] * Qm[0 * 2 + b] + QG[a * 2 + 1] * Qm[1 * 2 + b]);
        /* dSc = J^T H J ; dJ = 2 H J Sc */
        const double* J = P.J;
        double HJ[6];
        for (int a = 0; a < 2; ++a)
            for (int j = 0; j < 3; ++j) HJ[a * 3 + j] = H[a * 2 + 0] * J[0 * 3 + j] + H[a * 2 + 1] * J[1 * 3 + j];
        double dSc[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) dSc[a * 3 + b] = J[0 * 3 + a] * HJ[0 * 3 + b] + J[1 * 3 + a] * HJ[1 * 3 + b];
        double dJ[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double t = 0;
                for (int j = 0; j < 3; ++j) t += HJ[a * 3 + j] * P.Sc[j * 3 + b];
                dJ[a * 3 + b] = 2.0 * t;
            }
        /* J(p): J00 = fx/z, J02 = -fx xc / z (xc = x/z unless clamped), same for y */
        dp[2] += dJ[0] * (-c.fx / (z * z));
        dp[2] += dJ[4] * (-c.fy / (z * z));
        if (!P.clampx) {
            dp[0] += dJ[2] * (-c.fx / (z * z));
            dp[2] += dJ[2] * (2.0 * c.fx * x / (z * z * z));
        } else {
            double xcl = (x / z < 0) ? -c.limx : c.limx;
            dp[2] += dJ[2] * (c.fx * xcl / (z * z));
        }
        if (!P.clampy) {
            dp[1] += dJ[5] * (-c.fy / (z * z));
            dp[2] += dJ[5] * (2.0 * c.fy * y / (z * z * z));
        } else {
            double ycl = (y / z < 0) ? -c.limy : c.limy;
            dp[2] += dJ[5] * (c.fy * ycl / (z * z));
        }
        /* mu_w from p */
        double dmw[3];
        for (int j = 0; j < 3; ++j) dmw[j] = c.Rc[0 * 3 + j] * dp[0] + c.Rc[1 * 3 + j] * dp[1] + c.Rc[2 * 3 + j] * dp[2];
        /* Sc = Rc Sw Rc^T -> dSw = Rc^T dSc Rc */
        double T1[9], dSw[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) T1[a * 3 + b] = c.Rc[0 * 3 + a] * dSc[0 * 3 + b] + c.Rc[1 * 3 + a] * dSc[1 * 3 + b] + c.Rc[2 * 3 + a] * dSc[2 * 3 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) dSw[a * 3 + b] = T1[a * 3 + 0] * c.Rc[0 * 3 + b] + T1[a * 3 + 1] * c.Rc[1 * 3 + b] + T1[a * 3 + 2] * c.Rc[2 * 3 + b];
        /* Sw = M M^T, M = Rg diag(s): dM = (dSw + dSw^T) M */
        double M[9], dM[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a * 3 + b] = P.Rg[a * 3 + b] * P.s[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double t = 0;
                for (int j = 0; j < 3; ++j) t += (dSw[a * 3 + j] + dSw[j * 3 + a]) * M[j * 3 + b];
                dM[a * 3 + b] = t;
            }
        double ds[3] = {0, 0, 0}, dRg[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                ds[b] += dM[a * 3 + b] * P.Rg[a * 3 + b];
                dRg[a * 3 + b] = dM[a * 3 + b] * P.s[b];
            }
        /* Rg = Rk Rq -> dRq = Rk^T dRg */
        double dRq[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) dRq[a * 3 + b] = N->Rk[0 * 3 + a] * dRg[0 * 3 + b] + N->Rk[1 * 3 + a] * dRg[1 * 3 + b] + N->Rk[2 * 3 + a] * dRg[2 * 3 + b];
        /* R(qhat) -> qhat (w, x, y, z) */
        double q[4];
        for (int j = 0; j < 4; ++j) q[j] = sc->quats[4 * (size_t)i + j];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double w = q[0] / qn, qx = q[1] / qn, qy = q[2] / qn, qz = q[3] / qn;
        const double* G = dRq;
        double dqh[4];
        dqh[0] = 2.0 * (-qz * G[1] + qy * G[2] + qz * G[3] - qx * G[5] - qy * G[6] + qx * G[7]);
        dqh[1] = 2.0 * (qy * G[1] + qz * G[2] + qy * G[3] - 2 * qx * G[4] - w * G[5] + qz * G[6] + w * G[7] - 2 * qx * G[8]);
        dqh[2] = 2.0 * (-2 * qy * G[0] + qx * G[1] + w * G[2] + qx * G[3] + qz * G[5] - w * G[6] + qz * G[7] - 2 * qy * G[8]);
        dqh[3] = 2.0 * (-2 * qz * G[0] - w * G[1] + qx * G[2] + w * G[3] - 2 * qz * G[4] + qy * G[5] + qx * G[6] + qy * G[7]);
        /* qhat = q/|q| -> dq = (dqh - qhat (qhat.dqh)) / |q| */
        double qh[4] = {w, qx, qy, qz};
        double dd = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
        /* colour -> SH coefficients and view direction */
        double Y[OR_MAXK], dY[OR_MAXK * 3];
        or_sh_eval(L, P.dvec, Y, dY);
        double dkw[OR_MAXK * 3];
        for (int m = 0; m < K * 3; ++m) dkw[m] = 0.0;
        double ddir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            double gcol = gg[6 + ch];
            if (P.colpre[ch] < 0.0) gcol = 0.0;
            for (int m = 0; m < K; ++m) {
                dkw[m * 3 + ch] = gcol * Y[m];
                for (int j = 0; j < 3; ++j) ddir[j] += gcol * P.kw[m * 3 + ch] * dY[m * 3 + j];
            }
        }
        if (pg) {
            double M[9], *o = pg + 6 * (size_t)i;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    M[a * 3 + b] = dRg[a * 3 + 0] * P.Rg[b * 3 + 0] + dRg[a * 3 + 1] * P.Rg[b * 3 + 1] + dRg[a * 3 + 2] * P.Rg[b * 3 + 2];
            const double* m = P.mu_w;
            const double* cc = c.centre;
            o[0] = m[1] * dmw[2] - m[2] * dmw[1] + cc[1] * ddir[2] - cc[2] * ddir[1] + M[7] - M[5];
            o[1] = m[2] * dmw[0] - m[0] * dmw[2] + cc[2] * ddir[0] - cc[0] * ddir[2] + M[2] - M[6];
            o[2] = m[0] * dmw[1] - m[1] * dmw[0] + cc[0] * ddir[1] - cc[1] * ddir[0] + M[3] - M[1];
            for (int j = 0; j < 3; ++j) o[3 + j] = dmw[j] + ddir[j];
        }
        for (int j = 0; j < 3; ++j) dmw[j] += ddir[j];
        /* mu' = Rk mu + tk -> dmu = Rk^T dmu' */
        for (int j = 0; j < 3; ++j)
            d_means[3 * (size_t)i + j] += N->Rk[0 * 3 + j] * dmw[0] + N->Rk[1 * 3 + j] * dmw[1] + N->Rk[2 * 3 + j] * dmw[2];
        for (int j = 0; j < 3; ++j) d_scales[3 * (size_t)i + j] += ds[j];
        for (int j = 0; j < 4; ++j) d_quats[4 * (size_t)i + j] += (dqh[j] - qh[j] * dd) / qn;
        d_opac[i] += gg[5];
        /* k_w = D^T k -> dk = D dk_w */
        for (int m = 0; m < K; ++m)
            for (int ch = 0; ch < 3; ++ch) {
                double t = 0;
                for (int j = 0; j < K; ++j) t += N->D[m * K + j] * dkw[j * 3 + ch];
                d_sh[(size_t)i * K * 3 + m * 3 + ch] += t;
            }
    }
    if (pg) {
        for (int i = 0; i < sc->n; ++i)
            for (int j = 0; j < 6; ++j) d_pose[6 * (size_t)sc->node[i] + j] += pg[6 * (size_t)i + j];
        free(pg);
    }
    free(nd);
}

/* For pairs (Gaussian gidx[i], pixel (px[i], py[i])): the FP64 alpha before the 0.99 clamp,
   o exp(power), and the bound of an FP32 renderer's relative error of it (decision_bound). */
void or_alpha_bounds(const double* geo, int64_t npairs, const int32_t* gidx, const int32_t* px, const int32_t* py,
                     double* alpha, double* bound) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npairs; ++i) {
        const double* g = geo + (size_t)gidx[i] * GEO;
        const double dx = px[i] + 0.5 - g[0], dy = py[i] + 0.5 - g[1];
        const double power = -0.5 * (g[2] * dx * dx + g[4] * dy * dy) - g[3] * dx * dy;
        alpha[i] = g[5] * exp(power);
        bound[i] = decision_bound(g, dx, dy);
    }
}

/* Threads an OpenMP region of the oracle uses. */
int or_num_threads(void) { return omp_get_max_threads(); }

/* Flat-argument wrappers for ctypes. */
void or_keyspec_flat(int n, int sh_degree, const float* means, const float* scales, const float* quats,
                     const float* opac, const int32_t* node, int n_nodes,
                     const float* pose_R, const float* pose_t, const float* cam, int width, int height,
                     int tw, int th, int32_t* rect, uint32_t* zbits, int32_t* vis) {
    or_scene32 s;
    s.n = n; s.sh_degree = sh_degree; s.means = means; s.scales = scales; s.quats = quats; s.opac = opac;
    s.node = node; s.n_nodes = n_nodes; s.pose_R = pose_R; s.pose_t = pose_t;
    or_keyspec(&s, cam, width, height, tw, th, rect, zbits, vis);
}

static or_scene mk_scene(int n, int sh_degree, const double* means, const double* scales, const double* quats,
                         const double* opac, const double* sh, const int32_t* node, int n_nodes,
                         const double* pose_R, const double* pose_t) {
    or_scene s;
    s.n = n; s.sh_degree = sh_degree; s.means = means; s.scales = scales; s.quats = quats;
    s.opac = opac; s.sh = sh; s.node = node; s.n_nodes = n_nodes; s.pose_R = pose_R; s.pose_t = pose_t;
    return s;
}

void or_project_flat(int n, int sh_degree, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* sh, const int32_t* node, int n_nodes,
                     const double* pose_R, const double* pose_t, const double* cam, int width, int height,
                     double* geo) {
    or_scene s = mk_scene(n, sh_degree, means, scales, quats, opac, sh, node, n_nodes, pose_R, pose_t);
    or_project(&s, cam, width, height, geo);
}

void or_backward_project_flat(int n, int sh_degree, const double* means, const double* scales, const double* quats,
                              const double* opac, const double* sh, const int32_t* node, int n_nodes,
                              const double* pose_R, const double* pose_t, const double* cam, int width, int height,
                              const double* g2d, double* d_means, double* d_scales, double* d_quats,
                              double* d_opac, double* d_sh, double* d_pose) {
    or_scene s = mk_scene(n, sh_degree, means, scales, quats, opac, sh, node, n_nodes, pose_R, pose_t);
    or_backward_project(&s, cam, width, height, g2d, d_means, d_scales, d_quats, d_opac, d_sh, d_pose);
}
