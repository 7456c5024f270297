// Host-side derivation of the lattice weights and scale (Sec. IV).
//
// The paper obtains D2Q37 and D3Q107 by Gauss-Hermite quadrature: the
// weights w_i and the scale r (xi_i = r e_i) make the discrete sums
// reproduce the Hermite moments of the standard normal weight,
//
//     sum_i w_i He_a(xi_ix) He_b(xi_iy) [He_c(xi_iz)] = 1 if a=b=c=0, else 0,
//
// for all even (a, b, c) of total degree <= 8 (odd ones vanish by the
// lattice symmetry).  One condition per multi-index up to axis permutation
// gives G + 1 equations for the G group weights and r.  They are solved here
// by Newton's method in extended precision (x87 long double), started from
// the values printed in Tables I and II, and then rounded to double.  The
// probabilists' Hermite polynomials keep the system well conditioned
// (monomial moments would mix scales of 1 and 3^8 r^8).
#include <cmath>
#include <cstring>
#include <mutex>

#include "lbm_internal.h"

namespace lbm {
namespace {

typedef long double ld;

ld hermite(int n, ld x) {  // He_n(x): He_0 = 1, He_1 = x, He_{n+1} = x He_n - n He_{n-1}
    if (n == 0) return 1.0L;
    ld a = 1.0L, b = x;
    for (int k = 1; k < n; ++k) {
        ld c = x * b - (ld)k * a;
        a = b;
        b = c;
    }
    return b;
}

// Solve A x = b (n x n, row-major) by Gaussian elimination, partial pivoting.
bool solve(int n, ld* A, ld* b) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r * n + c]) > fabsl(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0L) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
            std::swap(b[c], b[p]);
        }
        for (int r = c + 1; r < n; ++r) {
            const ld f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        ld s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
    return true;
}

template <int D>
void derive(LatticeTables& t) {
    constexpr VelSet<D> vs = kVelSet<D>;
    constexpr int Q = VelSet<D>::Q, G = VelSet<D>::G, M = G + 1;
    // the paper's printed weights (Tables I and II) and scale: start values
    static const ld printed2[8] = {2.03916918e-1L, 1.27544846e-1L, 4.37537182e-2L,
                                   8.13659044e-3L, 9.40079914e-3L, 6.95051049e-4L,
                                   3.04298494e-5L, 2.81093762e-5L};
    static const ld printed3[10] = {1.603003550e-1L, 2.390868500e-2L, 4.169870315e-2L,
                                    5.166346780e-3L, 1.227117147e-2L, 2.676524495e-3L,
                                    9.685223338e-4L, 2.170763000e-5L, 2.453010230e-4L,
                                    1.417071270e-4L};
    // even multi-indices of degree <= 8, one per orbit (non-increasing)
    int alpha[M][3];
    int na = 0;
    for (int a = 0; a <= 8; a += 2)
        for (int b = 0; b <= a; b += 2)
            for (int c = 0; c <= (D == 3 ? b : 0); c += 2)
                if (a + b + c <= 8) {
                    alpha[na][0] = a;
                    alpha[na][1] = b;
                    alpha[na][2] = c;
                    ++na;
                }
    ld x[M];
    for (int g = 0; g < G; ++g) x[g] = D == 2 ? printed2[g] : printed3[g];
    x[G] = 1.19697977L;
    for (int it = 0; it < 60; ++it) {
        ld F[M], J[M * M];
        for (int m = 0; m < M; ++m) {
            F[m] = m == 0 ? -1.0L : 0.0L;  // alpha[0] = (0,0,0)
            for (int k = 0; k < M; ++k) J[m * M + k] = 0.0L;
        }
        const ld r = x[G];
        for (int i = 0; i < Q; ++i) {
            const int e[3] = {vs.v[i].x, vs.v[i].y, vs.v[i].z};
            const int g = vs.v[i].group;
            for (int m = 0; m < M; ++m) {
                ld he[3], dhe[3];
                for (int k = 0; k < 3; ++k) {
                    const int a = alpha[m][k];
                    he[k] = hermite(a, r * e[k]);
                    // d/dr He_a(r e) = a He_{a-1}(r e) e
                    dhe[k] = a > 0 ? (ld)a * hermite(a - 1, r * e[k]) * e[k] : 0.0L;
                }
                const ld prod = he[0] * he[1] * he[2];
                const ld dprod = dhe[0] * he[1] * he[2] + he[0] * dhe[1] * he[2] +
                                 he[0] * he[1] * dhe[2];
                F[m] += x[g] * prod;
                J[m * M + g] += prod;
                J[m * M + G] += x[g] * dprod;
            }
        }
        ld dx[M];
        for (int m = 0; m < M; ++m) dx[m] = -F[m];
        if (!solve(M, J, dx)) break;
        ld worst = 0.0L;
        for (int m = 0; m < M; ++m) {
            x[m] += dx[m];
            worst = fmaxl(worst, fabsl(dx[m]) / fabsl(x[m]));
        }
        if (worst < 1e-18L) break;
    }
    t.dim = D;
    t.q = Q;
    t.groups = G;
    t.r = (double)x[G];
    for (int g = 0; g < G; ++g) t.w_group[g] = (double)x[g];
    for (int i = 0; i < Q; ++i) {
        t.e[i][0] = (int8_t)vs.v[i].x;
        t.e[i][1] = (int8_t)vs.v[i].y;
        t.e[i][2] = (int8_t)vs.v[i].z;
        t.group[i] = vs.v[i].group;
        t.w[i] = t.w_group[vs.v[i].group];
    }
}

LatticeTables g_tables[2];
std::once_flag g_once;

}  // namespace

Physics physics_of(int dim, double delta, double tau_f, double tau_g, double dt,
                   bool energy_fix) {
    const LatticeTables& t = lattice_tables(dim);
    Physics ph;
    std::memset(&ph, 0, sizeof(ph));
    // lattice scheme: one lattice time step per step, rates 1/tau; the
    // finite-difference form: rates dt/tau and convection dt xi . grad
    const double step = dt > 0.0 ? dt : 1.0;
    ph.omega_f = step / tau_f;
    ph.omega_g = step / tau_g;
    ph.fd_cs = dt > 0.0 ? dt * t.r / 6.0 : 0.0;
    ph.fd_csf = (float)ph.fd_cs;
    // rates a_f / a_g = tau_g / tau_f in both forms
    ph.ec = energy_fix ? 1.0 - tau_g / tau_f : 0.0;
    ph.ecf = (float)ph.ec;
    ph.half_delta = 0.5 * delta;
    ph.inv_dof = 1.0 / (dim + delta);
    ph.r = t.r;
    for (int g = 0; g < t.groups; ++g) {
        ph.w[g] = t.w_group[g];
        ph.wf[g] = (float)t.w_group[g];
        ph.inv_wf[g] = (float)(1.0 / t.w_group[g]);
    }
    return ph;
}

// Population planes of the benchmark grids (256^3, 4096^2) are a large power
// of two bytes apart (a plane of 2^24 cells), and the 2Q plane streams of a
// step then start at one offset modulo every power of two up to that size.
// Moving the planes apart by a few kilobytes made the step faster on
// average over repeated allocations (each measured 2-15 times; single
// allocations vary by +-8% around these means): D3Q107 FP16 by 13%, FP32 by
// 4%, D2Q37 FP32 by 5%, FP16 and FP64 by 2-3%; D3Q107 FP64 by under 1%.  The
// pads are those means' best of the sizes tried.  Planes under 32 MiB
// (every smaller grid, the bulk of a serving pool) are only rounded up to
// 128 bytes, which keeps 16-byte row loads aligned.
namespace {
constexpr int64_t kPadFrom = int64_t(32) << 20;
constexpr int64_t kPad3[3] = {8320, 16896, 1280};   // D3Q107: 2-, 4-, 8-byte values
constexpr int64_t kPad2[3] = {33024, 16640, 8704};  // D2Q37
}  // namespace

int64_t plane_stride(int64_t N, size_t elem, int dim) {
    const int64_t bytes = (N * (int64_t)elem + 127) / 128 * 128;
    if (bytes < kPadFrom) return bytes / (int64_t)elem;
    const int k = elem == 2 ? 0 : (elem == 4 ? 1 : 2);
    return (bytes + (dim == 3 ? kPad3[k] : kPad2[k])) / (int64_t)elem;
}

const LatticeTables& lattice_tables(int dim) {
    std::call_once(g_once, [] {
        derive<2>(g_tables[0]);
        derive<3>(g_tables[1]);
    });
    return g_tables[dim == 2 ? 0 : 1];
}

}  // namespace lbm
