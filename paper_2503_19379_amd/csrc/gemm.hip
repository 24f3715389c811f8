// Matrix-core (MFMA) kernels of the Rayleigh-Ritz step of the block
// eigensolver (Section 5.1): the Gram products of the basis S = [X W P] and the
// block update with the Ritz coefficients.  FP64, v_mfma_f64_16x16x4f64.
//
// Operand layouts of the 16x16x4 FP64 MFMA (lane l of a 64-wide wave):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 r][l % 16], r = 0..3
// Complex products use three real products per 16x16x4 step:
//   conj(s) t : re = sr tr + si ti,  im = (sr - si)(tr + ti) - sr tr + si ti
//   s c       : re = sr cr - si ci,  im = (sr + si)(cr + ci) - sr cr - si ci
#include "common.h"
#include "solver.h"

namespace mfd {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Gram: for the K = 3mb basis columns S = V[:, :K] and AS = V[:, K:2K],
//   G_S = S^H S, G_A = S^H AS (both Hermitian: only 16x16 tiles touching the
//   upper triangle are formed; the reduction mirrors them).
// Workgroup w sums rows [w rows_per, (w+1) rows_per) into its own partial
// tile set; gram_reduce_kernel adds the partials in a fixed order.
// ---------------------------------------------------------------------------
constexpr int GM_KS = 16;       // rows per LDS slab
constexpr int GM_MAXT = 3;      // tiles per wave; one wave per GM_MAXT tiles, up to 16 waves

struct GramTiles {
    int n;                      // number of tiles
    short ti[80], tj[80];       // tile row (of G_S / G_A, 16 units) and column
    unsigned char half[80];     // 0: G_S, 1: G_A
};

__global__ __launch_bounds__(1024) void gram_mfma_kernel(const double2* __restrict__ V, size_t ld,
                                                                 size_t n, int K, size_t rows_per, GramTiles tl,
                                                                 double2* __restrict__ part) {
    extern __shared__ unsigned char smem_raw[];
    double2* slab = reinterpret_cast<double2*>(smem_raw);   // [GM_KS][2K]
    const int C2 = 2 * K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const size_t r0 = (size_t)blockIdx.x * rows_per;
    const size_t r1 = min(n, r0 + rows_per);
    const int my_n = (tl.n - wave + nwaves - 1) / nwaves;   // tiles wave, wave + nwaves, ...
    d4 acc[GM_MAXT][3];
#pragma unroll
    for (int t = 0; t < GM_MAXT; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[t][q] = d4{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;

    for (size_t s0 = r0; s0 < r1; s0 += GM_KS) {
        const int rows = (int)min((size_t)GM_KS, r1 - s0);
        for (int e = tid; e < GM_KS * C2; e += blockDim.x) {
            const int r = e % GM_KS, c = e / GM_KS;
            slab[r * C2 + c] = (r < rows) ? V[(size_t)c * ld + s0 + r] : mk<double2>(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < GM_KS; k0 += 4) {
            const double2* srow = slab + (k0 + lk) * C2;
#pragma unroll
            for (int t = 0; t < GM_MAXT; ++t) {
                if (t >= my_n) break;
                const int ti = wave + nwaves * t;
                const int i = tl.ti[ti] * 16 + li;
                const int j = tl.tj[ti] * 16 + li;
                const double2 a = (i < K) ? srow[i] : mk<double2>(0.0, 0.0);
                const double2 b = (j < K) ? srow[tl.half[ti] * K + j] : mk<double2>(0.0, 0.0);
                acc[t][0] = mfma64(a.x, b.x, acc[t][0]);
                acc[t][1] = mfma64(a.y, b.y, acc[t][1]);
                acc[t][2] = mfma64(a.x - a.y, b.x + b.y, acc[t][2]);
            }
        }
        __syncthreads();
    }
    // partial tiles: part[w][tile][16][16]
    double2* out = part + (size_t)blockIdx.x * tl.n * 256;
#pragma unroll
    for (int t = 0; t < GM_MAXT; ++t) {
        if (t >= my_n) break;
        const int ti = wave + nwaves * t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = lk + 4 * r, colj = li;
            const double t1 = acc[t][0][r], t2 = acc[t][1][r], t3 = acc[t][2][r];
            out[(size_t)ti * 256 + row * 16 + colj] = mk<double2>(t1 + t2, t3 - t1 + t2);
        }
    }
}

// G (K x 2K row-major) from the partial tiles; mirrors the lower triangles.
__global__ void gram_reduce_kernel(const double2* __restrict__ part, int nparts, int K, GramTiles tl,
                                   double2* __restrict__ G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tl.n * 256) return;
    const int t = e / 256, rc = e % 256;
    double sx = 0.0, sy = 0.0;
    for (int w = 0; w < nparts; ++w) {
        const double2 v = part[((size_t)w * tl.n + t) * 256 + rc];
        sx += v.x;
        sy += v.y;
    }
    const int i = tl.ti[t] * 16 + rc / 16, j = tl.tj[t] * 16 + rc % 16;
    if (i >= K || j >= K) return;
    const int off = tl.half[t] * K;
    if (i <= j) G[(size_t)i * 2 * K + off + j] = mk<double2>(sx, sy);
    if (i < j) G[(size_t)j * 2 * K + off + i] = mk<double2>(sx, -sy);
}

static GramTiles make_tiles(int K) {
    GramTiles tl;
    tl.n = 0;
    const int T = (K + 15) / 16;
    for (int h = 0; h < 2; ++h)
        for (int a = 0; a < T; ++a)
            for (int b = a; b < T; ++b) {
                tl.ti[tl.n] = (short)a;
                tl.tj[tl.n] = (short)b;
                tl.half[tl.n] = (unsigned char)h;
                ++tl.n;
            }
    return tl;
}

int gram_mfma_parts(size_t n) { return (int)std::min<size_t>(512, (n + 1023) / 1024); }

size_t gram_mfma_part_elems(int K, int nparts) {
    const int T = (K + 15) / 16;
    return (size_t)nparts * T * (T + 1) * 256;
}

hipError_t launch_gram_mfma(const void* V, size_t ld, size_t n, int K, int nparts, void* part, void* G,
                            hipStream_t s) {
    GramTiles tl = make_tiles(K);
    const int nwaves = (tl.n + GM_MAXT - 1) / GM_MAXT;
    if (nwaves > 16 || K > 64) return hipErrorInvalidValue;
    const size_t rows_per = ((n + nparts - 1) / nparts + GM_KS - 1) / GM_KS * GM_KS;
    const int nw = (int)((n + rows_per - 1) / rows_per);
    const size_t lds = (size_t)GM_KS * 2 * K * sizeof(double2);
    hipError_t e = hipFuncSetAttribute((const void*)gram_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_mfma_kernel, dim3(nw), dim3(64 * nwaves), lds, s, (const double2*)V, ld, n, K,
                       rows_per, tl, (double2*)part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((tl.n * 256 + 255) / 256), dim3(256), 0, s, (const double2*)part, nw,
                       K, tl, (double2*)G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Update with the Ritz coefficients C (K x mb, row-major), K = 3mb:
//   P' = [W P] C[mb:],  X' = P' + X C[:mb]  (and the same for AP', AX'),
//   R' = AX' - X' diag(theta),  column sums of |R'|^2 and |X'|^2.
// Output U = [X' | R' | P' | AX' | - | AP'].  Each wave owns 16-row strips;
// the coefficients sit in LDS as MFMA B fragments.
// ---------------------------------------------------------------------------
constexpr int UP_WAVES = 4;

template <int UP_MAXJ>   // mb <= 16 UP_MAXJ (16-column output tiles)
__global__ __launch_bounds__(64 * UP_WAVES) void update_mfma_kernel(const double2* __restrict__ V,
                                                                   double2* __restrict__ U, size_t ld, size_t n,
                                                                   int mb, const double2* __restrict__ Cg,
                                                                   const double* __restrict__ theta,
                                                                   double* __restrict__ npart) {
    extern __shared__ unsigned char smem_raw[];
    const int K = 3 * mb;
    const int KP = (K + 3) / 4 * 4;
    const int MP = UP_MAXJ * 16;
    double2* Cs = reinterpret_cast<double2*>(smem_raw);      // [KP][MP], zero padded
    double* red = reinterpret_cast<double*>(Cs + KP * MP);   // [UP_WAVES][2][MP]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < KP * MP; e += 64 * UP_WAVES) {
        const int k = e / MP, j = e % MP;
        Cs[e] = (k < K && j < mb) ? Cg[k * mb + j] : mk<double2>(0.0, 0.0);
    }
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    const int nj = (mb + 15) / 16;
    double th[UP_MAXJ];
    double nr[UP_MAXJ], nx[UP_MAXJ];
#pragma unroll
    for (int J = 0; J < UP_MAXJ; ++J) {
        const int j = 16 * J + li;
        th[J] = (j < mb) ? theta[j] : 0.0;
        nr[J] = nx[J] = 0.0;
    }
    const size_t nstrips = (n + 15) / 16;
    for (size_t st = (size_t)blockIdx.x * UP_WAVES + wave; st < nstrips; st += (size_t)gridDim.x * UP_WAVES) {
        const size_t row0 = st * 16;
        const size_t arow = row0 + li;          // A-fragment row of this lane
        const bool rok = arow < n;
        // accumulators: [J][chain X/AX][t1 t2 t3]
        d4 acc[UP_MAXJ][2][3];
#pragma unroll
        for (int J = 0; J < UP_MAXJ; ++J)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 3; ++q) acc[J][c][q] = d4{0.0, 0.0, 0.0, 0.0};
        // two passes over the basis columns: [mb, K) -> P', then [0, mb) -> X'
        for (int pass = 0; pass < 2; ++pass) {
            const int kb = pass == 0 ? mb : 0;
            const int ke = pass == 0 ? K : mb;
            for (int k0 = kb; k0 < ke; k0 += 4) {
                const int k = k0 + lk;
                double2 s = mk<double2>(0.0, 0.0), as = mk<double2>(0.0, 0.0);
                if (k < ke && rok) {
                    s = V[(size_t)k * ld + arow];
                    as = V[(size_t)(K + k) * ld + arow];
                }
                // rows of C: k (the wave's 4 k-rows) -- B fragment lane l: C[k0 + l/16][16 J + l%16];
                // k beyond ke reads C rows of the next range, but the A fragment there is zero.
#pragma unroll
                for (int J = 0; J < UP_MAXJ; ++J) {
                    if (J >= nj) break;
                    const double2 c = (k < ke) ? Cs[k * MP + 16 * J + li] : mk<double2>(0.0, 0.0);
                    const double cs = c.x + c.y;
                    acc[J][0][0] = mfma64(s.x, c.x, acc[J][0][0]);
                    acc[J][0][1] = mfma64(s.y, c.y, acc[J][0][1]);
                    acc[J][0][2] = mfma64(s.x + s.y, cs, acc[J][0][2]);
                    acc[J][1][0] = mfma64(as.x, c.x, acc[J][1][0]);
                    acc[J][1][1] = mfma64(as.y, c.y, acc[J][1][1]);
                    acc[J][1][2] = mfma64(as.x + as.y, cs, acc[J][1][2]);
                }
            }
            // write P' / AP' after the first pass, X' / AX' / R' after the second
#pragma unroll
            for (int J = 0; J < UP_MAXJ; ++J) {
                if (J >= nj) break;
                const int j = 16 * J + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t row = row0 + lk + 4 * r;
                    const double t1 = acc[J][0][0][r], t2 = acc[J][0][1][r], t3 = acc[J][0][2][r];
                    const double u1 = acc[J][1][0][r], u2 = acc[J][1][1][r], u3 = acc[J][1][2][r];
                    const double2 x = mk<double2>(t1 - t2, t3 - t1 - t2);
                    const double2 ax = mk<double2>(u1 - u2, u3 - u1 - u2);
                    if (j < mb && row < n) {
                        if (pass == 0) {
                            U[(size_t)(2 * mb + j) * ld + row] = x;
                            U[(size_t)(5 * mb + j) * ld + row] = ax;
                        } else {
                            const double2 res = mk<double2>(ax.x - th[J] * x.x, ax.y - th[J] * x.y);
                            U[(size_t)j * ld + row] = x;
                            U[(size_t)(3 * mb + j) * ld + row] = ax;
                            U[(size_t)(mb + j) * ld + row] = res;
                            nr[J] += cabs2(res);
                            nx[J] += cabs2(x);
                        }
                    }
                }
            }
        }
    }
    // column sums: lanes l, l+16, l+32, l+48 share column l % 16
#pragma unroll
    for (int J = 0; J < UP_MAXJ; ++J) {
        double a = nr[J], b = nx[J];
        a += __shfl_down(a, 32);
        b += __shfl_down(b, 32);
        a += __shfl_down(a, 16);
        b += __shfl_down(b, 16);
        if (lane < 16) {
            red[(wave * 2 + 0) * MP + 16 * J + lane] = a;
            red[(wave * 2 + 1) * MP + 16 * J + lane] = b;
        }
    }
    __syncthreads();
    if (tid < 2 * mb) {
        const int which = tid / mb, j = tid % mb;
        double s = 0.0;
        for (int w = 0; w < UP_WAVES; ++w) s += red[(w * 2 + which) * MP + j];
        npart[(size_t)blockIdx.x * 2 * mb + tid] = s;
    }
}

template <int MJ>
static hipError_t update_mj(const void* V, void* U, size_t ld, size_t n, int mb, const void* C, const double* theta,
                            int nparts, double* npart, hipStream_t s) {
    const int K = 3 * mb;
    const int KP = (K + 3) / 4 * 4;
    const size_t lds = (size_t)KP * MJ * 16 * sizeof(double2) + UP_WAVES * 2 * MJ * 16 * sizeof(double);
    auto kern = update_mfma_kernel<MJ>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nparts), dim3(64 * UP_WAVES), lds, s, (const double2*)V, (double2*)U, ld, n, mb,
                       (const double2*)C, theta, npart);
    return hipGetLastError();
}

hipError_t launch_update_mfma(const void* V, void* U, size_t ld, size_t n, int mb, const void* C,
                              const double* theta, int nparts, double* npart, double* norms, hipStream_t s) {
    hipError_t e;
    if (mb <= 16) e = update_mj<1>(V, U, ld, n, mb, C, theta, nparts, npart, s);
    else if (mb <= 32) e = update_mj<2>(V, U, ld, n, mb, C, theta, nparts, npart, s);
    else return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    return launch_reduce(npart, nparts, 2 * mb, norms, s);
}

}  // namespace mfd
