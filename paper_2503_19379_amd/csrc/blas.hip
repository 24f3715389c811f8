// Tall-skinny block algebra of the LOBPCG band solve (Section 5.1: the
// eigensolver minimises the Rayleigh quotient over span[X, W, P]) and the
// recompute check of Alg 4.1.
//
// Blocks are column-major n x j arrays of interleaved complex FP64, one
// column per band (the field layout [band][comp][z][y][x]).  The solver keeps
//   V = [X | W | P | AX | AW | AP]   (n x 6 mb)
// so that one Gram product G = V[:, :3mb]^H V covers both S^H S and S^H A S.
#include "common.h"
#include "internal.h"
#include "solver.h"

namespace mfd {

using C128 = double2;

// ---------------------------------------------------------------------------
// Gram:  Gpart[w] = V[rows of w, :P]^H V[rows of w, :Q]   (split over rows)
// ---------------------------------------------------------------------------
constexpr int GRAM_KS = 32;       // rows per LDS slab
constexpr int GRAM_TI = 5;        // P <= 16 * GRAM_TI
constexpr int GRAM_TJ = 8;        // Q <= 16 * GRAM_TJ

__global__ __launch_bounds__(256) void gram_kernel(const C128* __restrict__ V, size_t ld, size_t n, int P, int Q,
                                                   size_t rows_per, C128* __restrict__ part) {
    __shared__ C128 slab[GRAM_KS][16 * GRAM_TJ];
    const int tid = threadIdx.x;
    const int ti = tid & 15, tj = tid >> 4;
    const size_t r0 = (size_t)blockIdx.x * rows_per;
    const size_t r1 = min(n, r0 + rows_per);
    C128 acc[GRAM_TI][GRAM_TJ];
#pragma unroll
    for (int a = 0; a < GRAM_TI; ++a)
#pragma unroll
        for (int b = 0; b < GRAM_TJ; ++b) acc[a][b] = mk<C128>(0, 0);

    for (size_t s0 = r0; s0 < r1; s0 += GRAM_KS) {
        const int rows = (int)min((size_t)GRAM_KS, r1 - s0);
        for (int e = tid; e < GRAM_KS * Q; e += 256) {
            const int r = e % GRAM_KS, c = e / GRAM_KS;
            slab[r][c] = (r < rows) ? V[(size_t)c * ld + s0 + r] : mk<C128>(0, 0);
        }
        __syncthreads();
        for (int r = 0; r < rows; ++r) {
            C128 av[GRAM_TI], bv[GRAM_TJ];
#pragma unroll
            for (int a = 0; a < GRAM_TI; ++a) {
                const int i = ti + 16 * a;
                av[a] = (i < P) ? slab[r][i] : mk<C128>(0, 0);
            }
#pragma unroll
            for (int b = 0; b < GRAM_TJ; ++b) {
                const int j = tj + 16 * b;
                bv[b] = (j < Q) ? slab[r][j] : mk<C128>(0, 0);
            }
#pragma unroll
            for (int a = 0; a < GRAM_TI; ++a)
#pragma unroll
                for (int b = 0; b < GRAM_TJ; ++b) acc[a][b] = cfmac(acc[a][b], av[a], bv[b]);
        }
        __syncthreads();
    }
    C128* out = part + (size_t)blockIdx.x * P * Q;
#pragma unroll
    for (int a = 0; a < GRAM_TI; ++a)
#pragma unroll
        for (int b = 0; b < GRAM_TJ; ++b) {
            const int i = ti + 16 * a, j = tj + 16 * b;
            if (i < P && j < Q) out[i * Q + j] = acc[a][b];
        }
}

// out[c] = sum_w in[w * ncols + c] in a fixed order (deterministic): a
// workgroup owns CG columns; its 256 / CG thread rows stride over the parts
// and a tree in LDS combines them.
template <int CG>
__global__ __launch_bounds__(256) void reduce_parts_kernel(const double* __restrict__ in, int nparts, int ncols,
                                                           double* __restrict__ out) {
    constexpr int RG = 256 / CG;
    __shared__ double red[256];
    const int cl = threadIdx.x % CG, g = threadIdx.x / CG;
    const int c = blockIdx.x * CG + cl;
    double s = 0.0;
    if (c < ncols) {
        // eight loads in flight ahead of their adds; the adds keep the order
        // w = g, g + RG, ... so the sum does not depend on the batching
        int w = g;
        for (; w + 7 * RG < nparts; w += 8 * RG) {
            double t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = in[(size_t)(w + j * RG) * ncols + c];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += t[j];
        }
        for (; w < nparts; w += RG) s += in[(size_t)w * ncols + c];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = RG / 2; h > 0; h >>= 1) {
        if (g < h) red[threadIdx.x] += red[threadIdx.x + h * CG];
        __syncthreads();
    }
    if (g == 0 && c < ncols) out[c] = red[cl];
}

hipError_t launch_reduce(const double* parts, int nparts, int ncols, double* out, hipStream_t s) {
    if (ncols <= 128)
        hipLaunchKernelGGL(reduce_parts_kernel<1>, dim3(ncols), dim3(256), 0, s, parts, nparts, ncols, out);
    else
        hipLaunchKernelGGL(reduce_parts_kernel<32>, dim3((ncols + 31) / 32), dim3(256), 0, s, parts, nparts, ncols,
                           out);
    return hipGetLastError();
}

hipError_t launch_gram(const void* V, size_t ld, size_t n, int P, int Q, int nparts, void* part, void* G,
                       hipStream_t s) {
    if (P > 16 * GRAM_TI || Q > 16 * GRAM_TJ) return hipErrorInvalidValue;
    const size_t rows_per = (n + nparts - 1) / nparts;
    const int nw = (int)((n + rows_per - 1) / rows_per);
    hipLaunchKernelGGL(gram_kernel, dim3(nw), dim3(256), 0, s, (const C128*)V, ld, n, P, Q, rows_per, (C128*)part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce((const double*)part, nw, 2 * P * Q, (double*)G, s);
}

int gram_parts(size_t n) { return (int)std::min<size_t>(512, (n + 1023) / 1024); }

// ---------------------------------------------------------------------------
// Update: with C (3mb x mb) from the Rayleigh-Ritz step,
//   P' = [W P] C[mb:],  X' = P' + X C[:mb],  AP' = [AW AP] C[mb:],  AX' = AP' + AX C[:mb],
//   R' = AX' - X' diag(theta)
// written to U = [X' | R' | P' | AX' | - | AP'], plus per-workgroup partial
// sums of |R'_j|^2 and |X'_j|^2.
// ---------------------------------------------------------------------------
constexpr int UPD_MB = 32;

template <int MBT>
__global__ __launch_bounds__(256) void update_kernel(const C128* __restrict__ V, C128* __restrict__ U, size_t ld,
                                                     size_t n, int mb, const C128* __restrict__ Cg,
                                                     const double* __restrict__ theta, double* __restrict__ npart) {
    __shared__ C128 Cs[3 * MBT * MBT];
    __shared__ double th[MBT];
    __shared__ double red[2 * MBT][8];
    const int tid = threadIdx.x;
    const int K = 3 * mb;
    for (int e = tid; e < K * mb; e += 256) Cs[e] = Cg[e];   // row-major K x mb
    if (tid < mb) th[tid] = theta[tid];
    __syncthreads();
    double nr[MBT], nx[MBT];
#pragma unroll
    for (int r = 0; r < MBT; ++r) nr[r] = nx[r] = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + tid; i < n; i += stride) {
        C128 ax[MBT], aa[MBT];
#pragma unroll
        for (int r = 0; r < MBT; ++r) ax[r] = aa[r] = mk<C128>(0, 0);
        // P part: columns mb..3mb of S and of AS
        for (int j = mb; j < K; ++j) {
            const C128 s = V[(size_t)j * ld + i];
            const C128 as = V[(size_t)(K + j) * ld + i];
            const C128* cr = Cs + j * mb;
#pragma unroll
            for (int r = 0; r < MBT; ++r)
                if (r < mb) {
                    const C128 c = cr[r];
                    ax[r] = cfma(ax[r], s, c);
                    aa[r] = cfma(aa[r], as, c);
                }
        }
#pragma unroll
        for (int r = 0; r < MBT; ++r)
            if (r < mb) {
                U[(size_t)(2 * mb + r) * ld + i] = ax[r];
                U[(size_t)(5 * mb + r) * ld + i] = aa[r];
            }
        for (int j = 0; j < mb; ++j) {
            const C128 s = V[(size_t)j * ld + i];
            const C128 as = V[(size_t)(K + j) * ld + i];
            const C128* cr = Cs + j * mb;
#pragma unroll
            for (int r = 0; r < MBT; ++r)
                if (r < mb) {
                    const C128 c = cr[r];
                    ax[r] = cfma(ax[r], s, c);
                    aa[r] = cfma(aa[r], as, c);
                }
        }
#pragma unroll
        for (int r = 0; r < MBT; ++r)
            if (r < mb) {
                const C128 res = mk<C128>(aa[r].x - th[r] * ax[r].x, aa[r].y - th[r] * ax[r].y);
                U[(size_t)r * ld + i] = ax[r];
                U[(size_t)(3 * mb + r) * ld + i] = aa[r];
                U[(size_t)(mb + r) * ld + i] = res;
                nr[r] += cabs2(res);
                nx[r] += cabs2(ax[r]);
            }
    }
    // block reduction of the column norms (fixed order)
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int r = 0; r < MBT; ++r) {
        if (r >= mb) break;
        double a = nr[r], b = nx[r];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_down(a, o);
            b += __shfl_down(b, o);
        }
        if (lane == 0) { red[r][wid] = a; red[mb + r][wid] = b; }
    }
    __syncthreads();
    if (tid < 2 * mb) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[tid][w];
        npart[(size_t)blockIdx.x * 2 * mb + tid] = s;
    }
}

hipError_t launch_update(const void* V, void* U, size_t ld, size_t n, int mb, const void* C, const double* theta,
                         int nparts, double* npart, double* norms, hipStream_t s) {
    if (mb > UPD_MB) return hipErrorInvalidValue;
    if (mb <= 8)
        hipLaunchKernelGGL(update_kernel<8>, dim3(nparts), dim3(256), 0, s, (const C128*)V, (C128*)U, ld, n, mb,
                           (const C128*)C, theta, npart);
    else if (mb <= 16)
        hipLaunchKernelGGL(update_kernel<16>, dim3(nparts), dim3(256), 0, s, (const C128*)V, (C128*)U, ld, n, mb,
                           (const C128*)C, theta, npart);
    else if (mb <= 24)
        hipLaunchKernelGGL(update_kernel<24>, dim3(nparts), dim3(256), 0, s, (const C128*)V, (C128*)U, ld, n, mb,
                           (const C128*)C, theta, npart);
    else
        hipLaunchKernelGGL(update_kernel<32>, dim3(nparts), dim3(256), 0, s, (const C128*)V, (C128*)U, ld, n, mb,
                           (const C128*)C, theta, npart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(npart, nparts, 2 * mb, norms, s);
}

// ---------------------------------------------------------------------------
// Column statistics for the final check: dots[j] = (x_j^H x_j, Re x_j^H y_j);
// then res2[j] = |y_j - theta_j x_j|^2 with theta_j = Re(x^H y) / x^H x.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void colstats_kernel(const C128* __restrict__ X, const C128* __restrict__ Y,
                                                       size_t ld, size_t n, int nb, const double* __restrict__ theta,
                                                       double* __restrict__ part) {
    // blockIdx.y = column; theta == nullptr: pass 1 (dots), else pass 2 (residual norm)
    const int col = blockIdx.y;
    const C128* x = X + (size_t)col * ld;
    const C128* y = Y + (size_t)col * ld;
    double a = 0.0, b = 0.0;
    const double th = theta ? theta[col] : 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const C128 xv = x[i], yv = y[i];
        if (!theta) {
            a += cabs2(xv);
            b += xv.x * yv.x + xv.y * yv.y;
        } else {
            const double rx = yv.x - th * xv.x, ry = yv.y - th * xv.y;
            a += rx * rx + ry * ry;
        }
    }
    __shared__ double red[2][4];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o);
        b += __shfl_down(b, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { red[0][wid] = a; red[1][wid] = b; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[threadIdx.x][w];
        part[((size_t)blockIdx.x * nb + col) * 2 + threadIdx.x] = s;
    }
}

hipError_t launch_colstats(const void* X, const void* Y, size_t ld, size_t n, int nb, const double* theta,
                           int nparts, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(colstats_kernel, dim3(nparts, nb), dim3(256), 0, s, (const C128*)X, (const C128*)Y, ld, n, nb,
                       theta, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(part, nparts, 2 * nb, out, s);
}

// ---------------------------------------------------------------------------
// Residual refresh: R_j = AX_j - theta_j X_j (written as c64 or c128) and the
// per-workgroup column sums of |R_j|^2, |X_j|^2 (layout of the update's norms).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void residual_kernel(const C128* __restrict__ X, const C128* __restrict__ AX,
                                                       void* __restrict__ R, int r32, size_t ld, size_t n, int mb,
                                                       const double* __restrict__ theta, double* __restrict__ npart) {
    const int col = blockIdx.y;
    const double th = theta[col];
    const C128* x = X + (size_t)col * ld;
    const C128* ax = AX + (size_t)col * ld;
    double a = 0.0, b = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const C128 xv = x[i], yv = ax[i];
        const double rx = yv.x - th * xv.x, ry = yv.y - th * xv.y;
        if (r32) ((float2*)R)[(size_t)col * ld + i] = make_float2((float)rx, (float)ry);
        else ((C128*)R)[(size_t)col * ld + i] = mk<C128>(rx, ry);
        a += rx * rx + ry * ry;
        b += cabs2(xv);
    }
    __shared__ double red[2][4];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o);
        b += __shfl_down(b, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { red[0][wid] = a; red[1][wid] = b; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[threadIdx.x][w];
        npart[(size_t)blockIdx.x * 2 * mb + threadIdx.x * mb + col] = s;
    }
}

hipError_t launch_residual(const void* X, const void* AX, void* R, bool r32, size_t ld, size_t n, int mb,
                           const double* theta, int nparts, double* npart, double* norms, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(nparts, mb), dim3(256), 0, s, (const C128*)X, (const C128*)AX, R,
                       (int)r32, ld, n, mb, theta, npart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(npart, nparts, 2 * mb, norms, s);
}

// ---------------------------------------------------------------------------
// Alg 4.1, step 2: |M_0^(1/2) A' x|^2 per field, and |x|^2.
// ---------------------------------------------------------------------------
struct LamCoef {
    int K;
    double c[4], d[4];   // unit-step stencil
    double B[3][3];      // B[i][j]: weight of the difference along grid axis j in D_i
    double alpha[3];
};

__device__ __forceinline__ C128 lam_at(const C128* u, int N, int x, int y, int z, int axis, int off) {
    if (axis == 0) x = (x + off + 4 * N) % N;
    else if (axis == 1) y = (y + off + 4 * N) % N;
    else z = (z + off + 4 * N) % N;
    return u[((size_t)z * N + y) * N + x];
}

// (D_i' u)[r] = sum_j B_ij sum_s c_s (u[r - s e_j] - u[r + (s-1) e_j])
//               - i alpha_i sum_s d_s (u[r - s e_i] + u[r + (s-1) e_i])
__device__ __forceinline__ C128 lam_dadj(const LamCoef& w, const C128* u, int N, int x, int y, int z, int axis) {
    C128 diff = mk<C128>(0, 0), avg = mk<C128>(0, 0);
    for (int j = 0; j < 3; ++j) {
        const double bj = w.B[axis][j];
        if (bj == 0.0) continue;
        C128 dj = mk<C128>(0, 0);
        for (int s = 1; s <= w.K; ++s)
            dj = cadd(dj, cscale(csub(lam_at(u, N, x, y, z, j, -s), lam_at(u, N, x, y, z, j, s - 1)), w.c[s - 1]));
        diff = cadd(diff, cscale(dj, bj));
    }
    for (int s = 1; s <= w.K; ++s)
        avg = cadd(avg, cscale(cadd(lam_at(u, N, x, y, z, axis, -s), lam_at(u, N, x, y, z, axis, s - 1)), w.d[s - 1]));
    const double al = w.alpha[axis];
    return mk<C128>(diff.x + al * avg.y, diff.y - al * avg.x);
}

__global__ __launch_bounds__(256) void lambda_re_kernel(const C128* __restrict__ X, const double* __restrict__ mu,
                                                        int N, LamCoef w, int nb, double* __restrict__ part) {
    const int band = blockIdx.y;
    const size_t NN = (size_t)N * N, N3 = NN * N;
    const C128* v = X + (size_t)band * 3 * N3;
    double a = 0.0, b = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N3; i += (size_t)gridDim.x * 256) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / NN);
        const C128 v1 = v[i], v2 = v[N3 + i], v3 = v[2 * N3 + i];
        const C128 e1 = csub(lam_dadj(w, v + N3, N, x, y, z, 2), lam_dadj(w, v + 2 * N3, N, x, y, z, 1));
        const C128 e2 = csub(lam_dadj(w, v + 2 * N3, N, x, y, z, 0), lam_dadj(w, v, N, x, y, z, 2));
        const C128 e3 = csub(lam_dadj(w, v, N, x, y, z, 1), lam_dadj(w, v + N3, N, x, y, z, 0));
        a += mu[i] * cabs2(e1) + mu[N3 + i] * cabs2(e2) + mu[2 * N3 + i] * cabs2(e3);
        b += cabs2(v1) + cabs2(v2) + cabs2(v3);
    }
    __shared__ double red[2][4];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o);
        b += __shfl_down(b, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { red[0][wid] = a; red[1][wid] = b; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w2 = 0; w2 < 4; ++w2) s += red[threadIdx.x][w2];
        part[((size_t)blockIdx.x * nb + band) * 2 + threadIdx.x] = s;
    }
}

hipError_t launch_lambda_re(const OpParams& p, int nb, const void* X, const void* mu, double* partial, int nparts,
                            double* out, hipStream_t s) {
    LamCoef w;
    w.K = p.order / 2;
    double c[4], d[4];
    stencil_coefs(p.order, c, d);
    for (int q = 0; q < 4; ++q) {
        w.c[q] = c[q];
        w.d[q] = d[q];
    }
    for (int i = 0; i < 3; ++i) {
        w.alpha[i] = p.k[i];
        for (int j = 0; j < 3; ++j) w.B[i][j] = diff_weight(p, i, j);
    }
    hipLaunchKernelGGL(lambda_re_kernel, dim3(nparts, nb), dim3(256), 0, s, (const C128*)X, (const double*)mu, p.N,
                       w, nb, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partial, nparts, 2 * nb, out, s);
}

// ---------------------------------------------------------------------------
// Random start vectors: SplitMix64 (Steele, Lea, Flood 2014) on the counter
// (seed, index) gives two uniforms; Box-Muller turns them into N(0,1) for the
// real and imaginary parts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void fill_random_kernel(C128* __restrict__ X, size_t count, uint64_t seed) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed ^ splitmix64(2 * i));
        const uint64_t b = splitmix64(seed ^ splitmix64(2 * i + 1));
        const double u1 = ((a >> 11) + 1) * (1.0 / 9007199254740993.0);   // (0, 1]
        const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);         // [0, 1)
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        X[i] = mk<C128>(r * cs, r * sn);
    }
}

hipError_t launch_fill_random(void* X, size_t count, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(fill_random_kernel, dim3(1024), dim3(256), 0, s, (C128*)X, count, seed);
    return hipGetLastError();
}

__global__ void planewave_start_kernel(C128* __restrict__ X, int N, PlaneWaves pw, double noise) {
    const size_t N3 = (size_t)N * N * N, n = 3 * N3, count = n * (size_t)pw.mb;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i / n);
        const size_t rem = i % n;
        const int c = (int)(rem / N3);
        const size_t cell = rem % N3;
        const int x = (int)(cell % N), y = (int)((cell / N) % N), z = (int)(cell / ((size_t)N * N));
        // the phase m . r mod N in integers, then sincospi(2 t / N)
        long long t = ((long long)pw.m[j][0] * x + (long long)pw.m[j][1] * y + (long long)pw.m[j][2] * z) % N;
        if (t < 0) t += N;
        double sn, cs;
        sincospi(2.0 * (double)t / (double)N, &sn, &cs);
        const C128 a = pw.pol[j][c];
        const C128 r = X[i];
        X[i] = mk<C128>(a.x * cs - a.y * sn + noise * r.x, a.x * sn + a.y * cs + noise * r.y);
    }
}

hipError_t launch_planewave_start(void* X, int N, const PlaneWaves& pw, double noise, hipStream_t s) {
    if (pw.mb < 1 || pw.mb > 22) return hipErrorInvalidValue;
    hipLaunchKernelGGL(planewave_start_kernel, dim3(2048), dim3(256), 0, s, (C128*)X, N, pw, noise);
    return hipGetLastError();
}

// Y[:, j] = X[:, j] scaled to FP32 / from FP32 (mixed precision helpers)
__global__ void c128_to_c64_kernel(const C128* __restrict__ X, float2* __restrict__ Y, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const C128 v = X[i];
        Y[i] = make_float2((float)v.x, (float)v.y);
    }
}
__global__ void c64_to_c128_kernel(const float2* __restrict__ X, C128* __restrict__ Y, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const float2 v = X[i];
        Y[i] = mk<C128>((double)v.x, (double)v.y);
    }
}

hipError_t launch_convert(const void* X, void* Y, size_t count, bool to_c64, hipStream_t s) {
    if (to_c64)
        hipLaunchKernelGGL(c128_to_c64_kernel, dim3(2048), dim3(256), 0, s, (const C128*)X, (float2*)Y, count);
    else
        hipLaunchKernelGGL(c64_to_c128_kernel, dim3(2048), dim3(256), 0, s, (const float2*)X, (C128*)Y, count);
    return hipGetLastError();
}

}  // namespace mfd
