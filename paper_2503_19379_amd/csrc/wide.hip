// Two-pass MFD operator: orders 2K = 4, 6, 8 (Section 4.1.3, eq. (2kfdm),
// Table FD_1D) and general lattices (Section 4.2).  It forms the compensated
// operator w = A M_0 A' + gamma B'B v + c v with every one-dimensional
// difference and midpoint value replaced by its 2K-point symmetric stencil.
// With the unit-step difference and average along grid axis j, periodic,
//   (K_j u)[r]  = sum_s c_s (u[r+s] - u[r+1-s]),   (L_j u)[r]  = sum_s d_s (u[r+s] + u[r+1-s]),
//   (K_j' u)[r] = sum_s c_s (u[r-s] - u[r-1+s]),   (L_j' u)[r] = sum_s d_s (u[r-s] + u[r-1+s]),
// the derivative of Cartesian axis i is
//   D_i  = sum_j B_ij K_j  + i alpha_i L_i,   D_i' = sum_j B_ij K_j' - i alpha_i L_i'
// (D_i' the adjoint of D_i).  B = I / h on a cubic cell; on the lattice of A
// the grid is the unit cube of y = A^-1 x and B_ij = N (A^-1)_ji, while the
// average stays along grid axis i.  The operator is assembled as in eq.
// (discrete_2nd_block):
//   e = A'v : e1 = D3'v2 - D2'v3, e2 = D1'v3 - D3'v1, e3 = D2'v1 - D1'v2;  e <- mu e
//   q = B v = D1 v1 + D2 v2 + D3 v3
//   w1 = D2 e3 - D3 e2, w2 = D3 e1 - D1 e3, w3 = D1 e2 - D2 e1;  w_i += gamma D_i' q;  w += c v.
// Two passes over the block: pass 1 writes e and q of each band to a scratch
// buffer, pass 2 forms w.  One thread per cell; neighbours along y and z come
// through the caches.
#include "common.h"
#include "internal.h"

namespace mfd {

// Table FD_1D.  The table prints c_1 = 25/64 for K = 3; consistency of the
// derivative stencil (sum_s (2s - 1) c_s = 1) requires 75/64.
static const double kC[4][4] = {{1.0, 0, 0, 0},
                                {9.0 / 8.0, -1.0 / 24.0, 0, 0},
                                {75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0, 0},
                                {1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0}};
static const double kD[4][4] = {{0.5, 0, 0, 0},
                                {9.0 / 16.0, -1.0 / 16.0, 0, 0},
                                {75.0 / 128.0, -25.0 / 256.0, 3.0 / 256.0, 0},
                                {1225.0 / 2048.0, -245.0 / 2048.0, 49.0 / 2048.0, -5.0 / 2048.0}};

void stencil_coefs(int order, double c[4], double d[4]) {
    const int K = order / 2;
    for (int s = 0; s < 4; ++s) {
        c[s] = (K >= 1 && K <= 4) ? kC[K - 1][s] : 0.0;
        d[s] = (K >= 1 && K <= 4) ? kD[K - 1][s] : 0.0;
    }
}

template <class R>
struct WideCoef {
    int K;
    R c[4], d[4];   // unit-step stencil
    R B[3][3];      // B[i][j]: weight of the difference along grid axis j in D_i
    R alpha[3];
};

// u: one component field [z][y][x]; (x, y, z) the cell; axis 0 = x, 1 = y, 2 = z.
// |off| <= K <= 4 <= N, so one conditional wrap keeps the index periodic;
// N^3 <= 128^3 fits a 32-bit index.
__device__ __forceinline__ int wrap(int c, int N) {
    c += (c < 0) ? N : 0;
    return c - ((c >= N) ? N : 0);
}

template <class R, class T>
__device__ __forceinline__ cplx<R> ld_shift(const T* u, int N, int x, int y, int z, int axis, int off) {
    if (axis == 0) x = wrap(x + off, N);
    else if (axis == 1) y = wrap(y + off, N);
    else z = wrap(z + off, N);
    const T v = u[(z * N + y) * N + x];
    return mk<cplx<R>>(v.x, v.y);
}

// sum_j B[axis][j] sum_s c_s (u[r + sg s e_j] - u[r + sg (1 - s) e_j]) + i sg alpha_axis
//   sum_s d_s (u[r + sg s e_axis] + u[r + sg (1 - s) e_axis]); sg = +1 gives D, sg = -1 gives D'.
// KC = 1: order 2 with every loop unrolled (the neighbour loads of a cell are
// then shared between the D_i that use them); KC = 0: K from w.
template <int SG, int KC, class R, class T>
__device__ __forceinline__ cplx<R> Dapply(const WideCoef<R>& w, const T* u, int N, int x, int y, int z, int axis) {
    const int K = KC ? KC : w.K;
    cplx<R> diff = mk<cplx<R>>(0, 0), avg = mk<cplx<R>>(0, 0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const R bj = w.B[axis][j];
        if (bj == (R)0) continue;
        cplx<R> dj = mk<cplx<R>>(0, 0);
        for (int s = 1; s <= K; ++s) {
            const cplx<R> a = ld_shift<R>(u, N, x, y, z, j, SG * s), b = ld_shift<R>(u, N, x, y, z, j, SG * (1 - s));
            dj = cadd(dj, cscale(csub(a, b), w.c[s - 1]));
        }
        diff = cadd(diff, cscale(dj, bj));
    }
    for (int s = 1; s <= K; ++s) {
        const cplx<R> a = ld_shift<R>(u, N, x, y, z, axis, SG * s), b = ld_shift<R>(u, N, x, y, z, axis, SG * (1 - s));
        avg = cadd(avg, cscale(cadd(a, b), w.d[s - 1]));
    }
    const R al = SG * w.alpha[axis];
    return mk<cplx<R>>(diff.x - al * avg.y, diff.y + al * avg.x);   // diff + i sg alpha avg
}

template <int KC, class R, class T>
__device__ __forceinline__ cplx<R> Dfwd(const WideCoef<R>& w, const T* u, int N, int x, int y, int z, int axis) {
    return Dapply<1, KC>(w, u, N, x, y, z, axis);
}

template <int KC, class R, class T>
__device__ __forceinline__ cplx<R> Dadj(const WideCoef<R>& w, const T* u, int N, int x, int y, int z, int axis) {
    return Dapply<-1, KC>(w, u, N, x, y, z, axis);
}

// pass 1: T[b] = [mu_1 e1, mu_2 e2, mu_3 e3, q] of field fl(b0 + b)
template <class R, class S, int KC>
__global__ __launch_bounds__(256) void wide_pass1_kernel(const cplx<S>* __restrict__ X, cplx<R>* __restrict__ T,
                                                         const R* __restrict__ mu, int N, int b0, int nb,
                                                         WideCoef<R> w, FieldList fl) {
    const int N3 = N * N * N;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= N3 || b >= nb) return;
    const int x = i % N, y = (i / N) % N, z = i / (N * N);
    const cplx<S>* v = X + (size_t)fl(b0 + b) * 3 * N3;
    const cplx<S>*v1 = v, *v2 = v + N3, *v3 = v + 2 * N3;
    const cplx<R> e1 = csub(Dadj<KC>(w, v2, N, x, y, z, 2), Dadj<KC>(w, v3, N, x, y, z, 1));
    const cplx<R> e2 = csub(Dadj<KC>(w, v3, N, x, y, z, 0), Dadj<KC>(w, v1, N, x, y, z, 2));
    const cplx<R> e3 = csub(Dadj<KC>(w, v1, N, x, y, z, 1), Dadj<KC>(w, v2, N, x, y, z, 0));
    const cplx<R> q = cadd(cadd(Dfwd<KC>(w, v1, N, x, y, z, 0), Dfwd<KC>(w, v2, N, x, y, z, 1)), Dfwd<KC>(w, v3, N, x, y, z, 2));
    cplx<R>* t = T + (size_t)b * 4 * N3;
    t[i] = cscale(e1, mu[i]);
    t[N3 + i] = cscale(e2, mu[N3 + i]);
    t[2 * N3 + i] = cscale(e3, mu[2 * N3 + i]);
    t[3 * N3 + i] = q;
}

// pass 2: Y = A e + gamma B' q + shift X
template <class R, class S, int KC>
__global__ __launch_bounds__(256) void wide_pass2_kernel(const cplx<S>* __restrict__ X, const cplx<R>* __restrict__ T,
                                                         cplx<S>* __restrict__ Y, int N, int b0, int nb,
                                                         WideCoef<R> w, R gamma, R shift, FieldList fl) {
    const int N3 = N * N * N;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= N3 || b >= nb) return;
    const int x = i % N, y = (i / N) % N, z = i / (N * N);
    const cplx<R>* t = T + (size_t)b * 4 * N3;
    const cplx<R>*e1 = t, *e2 = t + N3, *e3 = t + 2 * N3, *q = t + 3 * N3;
    const size_t f = (size_t)fl(b0 + b) * 3 * N3;
    const cplx<S>* v = X + f;
    cplx<S>* out = Y + f;
    cplx<R> w1 = csub(Dfwd<KC>(w, e3, N, x, y, z, 1), Dfwd<KC>(w, e2, N, x, y, z, 2));
    cplx<R> w2 = csub(Dfwd<KC>(w, e1, N, x, y, z, 2), Dfwd<KC>(w, e3, N, x, y, z, 0));
    cplx<R> w3 = csub(Dfwd<KC>(w, e2, N, x, y, z, 0), Dfwd<KC>(w, e1, N, x, y, z, 1));
    w1 = cadd(w1, cscale(Dadj<KC>(w, q, N, x, y, z, 0), gamma));
    w2 = cadd(w2, cscale(Dadj<KC>(w, q, N, x, y, z, 1), gamma));
    w3 = cadd(w3, cscale(Dadj<KC>(w, q, N, x, y, z, 2), gamma));
    const cplx<S> a1 = v[i], a2 = v[N3 + i], a3 = v[2 * N3 + i];
    out[i] = mk<cplx<S>>(w1.x + shift * (R)a1.x, w1.y + shift * (R)a1.y);
    out[N3 + i] = mk<cplx<S>>(w2.x + shift * (R)a2.x, w2.y + shift * (R)a2.y);
    out[2 * N3 + i] = mk<cplx<S>>(w3.x + shift * (R)a3.x, w3.y + shift * (R)a3.y);
}

template <class R, class S>
hipError_t launch_wide(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                       const FieldList& fl) {
    if (p.lattice && p.order == 2) return launch_lattice<R, S>(p, nb, X, Y, mu, s, fl);
    if (!p.wtmp || p.wtmp_bands < 1) return hipErrorInvalidValue;
    WideCoef<R> w;
    w.K = p.order / 2;
    double c[4], d[4];
    stencil_coefs(p.order, c, d);
    for (int q = 0; q < 4; ++q) {
        w.c[q] = (R)c[q];
        w.d[q] = (R)d[q];
    }
    for (int a = 0; a < 3; ++a) {
        w.alpha[a] = (R)p.k[a];
        for (int j = 0; j < 3; ++j) w.B[a][j] = (R)diff_weight(p, a, j);
    }
    const size_t N3 = (size_t)p.N * p.N * p.N;
    const unsigned gx = (unsigned)((N3 + 255) / 256);
    cplx<R>* T = (cplx<R>*)p.wtmp;
    auto k1 = (w.K == 1) ? wide_pass1_kernel<R, S, 1> : wide_pass1_kernel<R, S, 0>;
    auto k2 = (w.K == 1) ? wide_pass2_kernel<R, S, 1> : wide_pass2_kernel<R, S, 0>;
    for (int b0 = 0; b0 < nb; b0 += p.wtmp_bands) {
        const int nc = std::min(nb - b0, p.wtmp_bands);
        hipLaunchKernelGGL(k1, dim3(gx, nc), dim3(256), 0, s, (const cplx<S>*)X, T, (const R*)mu, p.N, b0, nc, w,
                           fl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k2, dim3(gx, nc), dim3(256), 0, s, (const cplx<S>*)X, (const cplx<R>*)T, (cplx<S>*)Y,
                           p.N, b0, nc, w, (R)p.gamma, (R)p.shift, fl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_wide<float, float>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                              const FieldList&);
template hipError_t launch_wide<double, double>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                                const FieldList&);
template hipError_t launch_wide<double, float>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                               const FieldList&);

}  // namespace mfd
