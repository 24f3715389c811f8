// Hard locking for the last iterations of a k-point (the block eigensolver of
// Section 5.1): once at most LK_NA bands still iterate, the converged bands'
// vectors X_L are frozen and left out of the Rayleigh-Ritz basis, the new
// search directions are made orthogonal to them, and the update touches only
// the bands still iterating.  Three kernels, all bound by HBM:
//   lock_coef:   c = X_L^H Y                  (per-workgroup partial sums)
//   lock_apply:  Y -= X_L c  (and Z -= A X_L c, keeping Z = A Y)
//   lock_update: the block update over the basis [X_A W P] of the bands A
//                still iterating (X', AX', R', P', AP' of those bands only)
// Y and Z are W (and AW) or P (and AP) columns; in mixed precision they are
// stored in FP32 and computed on in FP64.
#include "common.h"
#include "solver.h"

namespace mfd {

constexpr int LK_NT = 256;
constexpr int LK_TR = 32;   // rows per LDS tile of lock_coef

// Workgroup barrier that orders LDS only: the next tile's global loads stay
// in flight across it (a full barrier would wait for them too).
__device__ __forceinline__ void lk_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// part[w][l * nt + t] = sum over the rows of workgroup w of conj(X_l) Y_t.
// Tiles of LK_TR rows pass through LDS; the next tile's loads are issued
// before the current tile's products.  Each load slot q reads one column
// for the whole kernel (X_L slots first, then one Y slot), so its address is
// set once before the tile loop and every load in the loop is unconditional:
// no load waits for another.
constexpr int LK_QX = (LK_TR * LK_MAXL + LK_NT - 1) / LK_NT;   // X_L slots per thread
static_assert(LK_TR * LK_MAXT == LK_NT, "one Y slot per thread");
__global__ __launch_bounds__(LK_NT) void lock_coef_kernel(LockCols c, const double2* __restrict__ V,
                                                          const float2* __restrict__ V32, size_t ld, size_t n,
                                                          size_t rows_per, double2* __restrict__ part) {
    __shared__ double2 xs[LK_TR][LK_MAXL];
    __shared__ double2 ys[LK_TR][LK_MAXT];
    const int tid = threadIdx.x;
    const int nl = c.nl, nt = c.nt;
    const size_t r0 = (size_t)blockIdx.x * rows_per;
    const size_t r1 = min(n, r0 + rows_per);
    const int p = tid, l = p / max(nt, 1), t = p % max(nt, 1);
    const bool mine = p < nl * nt;
    double2 acc = mk<double2>(0.0, 0.0);
    // slot q of X_L: element tid + q LK_NT = row r (its low bits) of column
    // xcol[q] (clamped to the last column, stored only when in range); the
    // Y slot: row r of column ycol
    const int r = tid % LK_TR;
    const double2* xp[LK_QX];
#pragma unroll
    for (int q = 0; q < LK_QX; ++q) xp[q] = V + (size_t)c.xc[min((tid + q * LK_NT) / LK_TR, nl - 1)] * ld;
    // Y is read as two 8-byte halves of an element of es bytes (an FP32
    // element's second half is its first again), so that its load does not
    // depend on the precision either
    const int ycol = min(tid / LK_TR, nt - 1);
    const bool y32 = c.y32 != 0;
    const size_t es = y32 ? sizeof(float2) : sizeof(double2);
    const char* yp = y32 ? (const char*)(V32 + (size_t)c.yc[ycol] * ld) : (const char*)(V + (size_t)c.yc[ycol] * ld);
    double2 vx[LK_QX];
    uint2 ylo = make_uint2(0u, 0u), yhi = make_uint2(0u, 0u);
    auto load = [&](size_t s0) {
        const size_t row = min(s0 + r, r1 - 1);
#pragma unroll
        for (int q = 0; q < LK_QX; ++q) vx[q] = xp[q][row];
        const char* e = yp + row * es;
        ylo = *(const uint2*)e;
        yhi = *(const uint2*)(e + (es - sizeof(uint2)));
    };
    if (r0 < r1) load(r0);
    for (size_t s0 = r0; s0 < r1; s0 += LK_TR) {
        const bool live = s0 + r < r1;
#pragma unroll
        for (int q = 0; q < LK_QX; ++q) {
            const int col = (tid + q * LK_NT) / LK_TR;
            if (col < nl) xs[r][col] = live ? vx[q] : mk<double2>(0.0, 0.0);
        }
        if (tid / LK_TR < nt) {
            const double2 w = y32 ? mk<double2>((double)__uint_as_float(ylo.x), (double)__uint_as_float(ylo.y))
                                  : mk<double2>(__hiloint2double(ylo.y, ylo.x), __hiloint2double(yhi.y, yhi.x));
            ys[r][ycol] = live ? w : mk<double2>(0.0, 0.0);
        }
        lk_lds_barrier();
        if (s0 + LK_TR < r1) load(s0 + LK_TR);
        if (mine)
            for (int k = 0; k < LK_TR; ++k) acc = cfmac(acc, xs[k][l], ys[k][t]);
        lk_lds_barrier();
    }
    if (mine) part[(size_t)blockIdx.x * nl * nt + p] = acc;
}

// Y_t -= sum_l X_l coef[l][t]; with c.zpair also Z_t -= sum_l AX_l coef[l][t]
__global__ __launch_bounds__(LK_NT) void lock_apply_kernel(LockCols c, const double2* __restrict__ coef,
                                                           double2* __restrict__ V, float2* __restrict__ V32,
                                                           size_t ld, size_t n) {
    __shared__ double2 cf[LK_MAXL * LK_MAXT];
    const int nl = c.nl, nt = c.nt;
    for (int e = threadIdx.x; e < nl * nt; e += LK_NT) cf[e] = coef[e];
    __syncthreads();
    for (size_t row = (size_t)blockIdx.x * LK_NT + threadIdx.x; row < n; row += (size_t)gridDim.x * LK_NT) {
        for (int pass = 0; pass < (c.zpair ? 2 : 1); ++pass) {
            double2 acc[LK_MAXT];
#pragma unroll
            for (int t = 0; t < LK_MAXT; ++t) acc[t] = mk<double2>(0.0, 0.0);
            for (int l = 0; l < nl; ++l) {
                const double2 x = V[(size_t)(pass ? c.axc[l] : c.xc[l]) * ld + row];
#pragma unroll
                for (int t = 0; t < LK_MAXT; ++t)
                    if (t < nt) acc[t] = cfma(acc[t], x, cf[l * nt + t]);
            }
#pragma unroll
            for (int t = 0; t < LK_MAXT; ++t) {
                if (t >= nt) continue;
                const size_t o = (size_t)(pass ? c.zc[t] : c.yc[t]) * ld + row;
                if (c.y32) {
                    const float2 y = V32[o];
                    V32[o] = make_float2((float)((double)y.x - acc[t].x), (float)((double)y.y - acc[t].y));
                } else {
                    V[o] = csub(V[o], acc[t]);
                }
            }
        }
    }
}

// The update over the basis S = [X_A W_A P] (K columns) and AS: for output t
// (band act[t]) X'_t = S C[:, t], P'_t = the W, P part of it, the same for
// the images; R'_t = AX'_t - theta_t X'_t.  Norm partials |R'_t|^2, |X'_t|^2.
// One row per thread; the basis columns are read in chunks of LK_CH, every
// load of a chunk issued before its products (the column index is clamped
// and C's rows past K are zero).
// NA: the outputs held in registers (4 or LK_NA), so that small sets of
// iterating bands run at a higher occupancy.
constexpr int LK_CH = 8;
template <int NA>
__global__ __launch_bounds__(LK_NT) void lock_update_kernel(LockBasis b, const double2* __restrict__ V,
                                                            const float2* __restrict__ V32, double2* __restrict__ U,
                                                            float2* __restrict__ U32, size_t ld, size_t n,
                                                            const double2* __restrict__ Cg,
                                                            const double* __restrict__ theta,
                                                            double* __restrict__ npart) {
    constexpr int KP = (3 * NA + LK_CH - 1) / LK_CH * LK_CH;   // basis rows held: K <= 3 NA, whole chunks
    __shared__ double2 cs[KP * NA];   // C, rows past K and columns past na zero
    // basis column k (chain 0) and its image (chain 1): the byte offset of its
    // V or V32 column from V, and log2 of its element size (3 for FP32, 4 for
    // FP64); every load goes through V, so it stays a global load
    __shared__ long long boff[2][KP];
    __shared__ int esh[KP];
    __shared__ double th[NA];
    __shared__ double red[LK_NT / 64][2 * NA];
    const int na = b.na, K = b.K, mb = b.mb;
    for (int e = threadIdx.x; e < KP * NA; e += LK_NT) {
        const int k = e / NA, t = e % NA;
        cs[e] = (k < K && t < na) ? Cg[(size_t)k * na + t] : mk<double2>(0.0, 0.0);
    }
    if (threadIdx.x < KP) {
        const int k = min((int)threadIdx.x, K - 1);
        const bool h = (b.f32 >> k) & 1ull;
        const char* v0 = (const char*)V;
        boff[0][threadIdx.x] = h ? (const char*)(V32 + (size_t)b.sc[k] * ld) - v0 : (const char*)(V + (size_t)b.sc[k] * ld) - v0;
        boff[1][threadIdx.x] = h ? (const char*)(V32 + (size_t)b.ic[k] * ld) - v0 : (const char*)(V + (size_t)b.ic[k] * ld) - v0;
        esh[threadIdx.x] = h ? 3 : 4;
    }
    if (threadIdx.x < NA) th[threadIdx.x] = threadIdx.x < (unsigned)na ? theta[threadIdx.x] : 0.0;
    __shared__ int band[NA];
    if (threadIdx.x < NA) band[threadIdx.x] = b.act[threadIdx.x < (unsigned)na ? threadIdx.x : 0];
    __syncthreads();
    double nr[NA], nx[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) nr[t] = nx[t] = 0.0;
    const int nch = (K + LK_CH - 1) / LK_CH;
    for (size_t row = (size_t)blockIdx.x * LK_NT + threadIdx.x; row < n; row += (size_t)gridDim.x * LK_NT) {
        double2 xo[NA];
#pragma unroll 1
        for (int ch = 0; ch < 2; ++ch) {
            double2 ax[NA], ap[NA];
#pragma unroll
            for (int t = 0; t < NA; ++t) ax[t] = ap[t] = mk<double2>(0.0, 0.0);
#pragma unroll 1
            for (int c0 = 0; c0 < nch * LK_CH; c0 += LK_CH) {
                // every column read as two 8-byte halves (an FP32 element's
                // second half is its first again): the chunk's loads do not
                // depend on the precision and none waits for another
                uint2 lo[LK_CH], hi[LK_CH];
                bool h32[LK_CH];
#pragma unroll
                for (int q = 0; q < LK_CH; ++q) {
                    const int k = c0 + q, sh = esh[k];
                    const char* e = (const char*)V + boff[ch][k] + (row << sh);
                    h32[q] = sh == 3;
                    lo[q] = *(const uint2*)e;
                    hi[q] = *(const uint2*)(e + ((sh - 3) << 3));
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the chunk's loads ahead of its products
                double2 sv[LK_CH];
#pragma unroll
                for (int q = 0; q < LK_CH; ++q) {
                    const double fr = (double)__uint_as_float(lo[q].x), fi = (double)__uint_as_float(lo[q].y);
                    const double dr = __hiloint2double(lo[q].y, lo[q].x), di = __hiloint2double(hi[q].y, hi[q].x);
                    sv[q].x = h32[q] ? fr : dr;
                    sv[q].y = h32[q] ? fi : di;
                }
#pragma unroll
                for (int q = 0; q < LK_CH; ++q) {
                    const int k = c0 + q;
#pragma unroll
                    for (int t = 0; t < NA; ++t) {
                        const double2 cv = cs[k * NA + t];
                        ax[t] = cfma(ax[t], sv[q], cv);
                        if (k >= na) ap[t] = cfma(ap[t], sv[q], cv);   // a W or P column
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                if (t >= na) continue;
                const int bj = band[t];
                if (ch == 0) {
                    xo[t] = ax[t];
                    U[(size_t)bj * ld + row] = ax[t];
                    if (U32) U32[(size_t)(2 * mb + bj) * ld + row] = make_float2((float)ap[t].x, (float)ap[t].y);
                    else U[(size_t)(2 * mb + bj) * ld + row] = ap[t];
                } else {
                    U[(size_t)(3 * mb + bj) * ld + row] = ax[t];
                    const double2 res = mk<double2>(ax[t].x - th[t] * xo[t].x, ax[t].y - th[t] * xo[t].y);
                    if (U32) {
                        U32[(size_t)(mb + bj) * ld + row] = make_float2((float)res.x, (float)res.y);
                        U32[(size_t)(5 * mb + bj) * ld + row] = make_float2((float)ap[t].x, (float)ap[t].y);
                    } else {
                        U[(size_t)(mb + bj) * ld + row] = res;
                        U[(size_t)(5 * mb + bj) * ld + row] = ap[t];
                    }
                    nr[t] += cabs2(res);
                    nx[t] += cabs2(xo[t]);
                }
            }
        }
    }
    // per-workgroup sums: lanes by shuffles, then the waves in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
        double a = nr[t], c = nx[t];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_down(a, o);
            c += __shfl_down(c, o);
        }
        if (lane == 0) {
            red[wave][t] = a;
            red[wave][NA + t] = c;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)(2 * na)) {
        const int which = threadIdx.x / na, t = threadIdx.x % na;
        double v = 0.0;
        for (int w = 0; w < LK_NT / 64; ++w) v += red[w][which * NA + t];
        npart[(size_t)blockIdx.x * 2 * na + threadIdx.x] = v;
    }
}

// First stage of the fixed-order sum of many partials: group g of LK_GS
// consecutive partials into tmp[g] (one thread per column); the groups are
// then summed by launch_reduce.
constexpr int LK_GS = 64;
__global__ __launch_bounds__(64) void lock_sum_kernel(const double* __restrict__ in, int nparts, int ncols,
                                                      double* __restrict__ tmp) {
    const int c = blockIdx.x * 64 + threadIdx.x, g = blockIdx.y;
    if (c >= ncols) return;
    const int w1 = min(nparts, (g + 1) * LK_GS);
    double v = 0.0;
    int w = g * LK_GS;
    for (; w + 8 <= w1; w += 8) {   // eight loads in flight, added in order
        double t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = in[(size_t)(w + j) * ncols + c];
#pragma unroll
        for (int j = 0; j < 8; ++j) v += t[j];
    }
    for (; w < w1; ++w) v += in[(size_t)w * ncols + c];
    tmp[(size_t)g * ncols + c] = v;
}

hipError_t launch_lock_coef(const LockCols& c, const void* V, const void* V32, size_t ld, size_t n, int nparts,
                            void* part, void* coef, hipStream_t s) {
    if (c.nl < 1 || c.nl > LK_MAXL || c.nt < 1 || c.nt > LK_MAXT || c.nl * c.nt > LK_NT || nparts < 1 || !n)
        return hipErrorInvalidValue;
    const size_t rows_per = ((n + nparts - 1) / nparts + LK_TR - 1) / LK_TR * LK_TR;
    const int nw = (int)((n + rows_per - 1) / rows_per);
    hipLaunchKernelGGL(lock_coef_kernel, dim3(nw), dim3(LK_NT), 0, s, c, (const double2*)V, (const float2*)V32, ld,
                       n, rows_per, (double2*)part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // part holds nparts + nparts / LK_GS + 1 partial sets: the group sums
    // follow the workgroups' partials
    const int ncols = 2 * c.nl * c.nt, ng = (nw + LK_GS - 1) / LK_GS;
    double* tmp = (double*)part + (size_t)nw * ncols;
    hipLaunchKernelGGL(lock_sum_kernel, dim3((ncols + 63) / 64, ng), dim3(64), 0, s, (const double*)part, nw, ncols,
                       tmp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_reduce(tmp, ng, ncols, (double*)coef, s);
}

hipError_t launch_lock_apply(const LockCols& c, const void* coef, void* V, void* V32, size_t ld, size_t n,
                             int nblocks, hipStream_t s) {
    if (c.nl < 1 || c.nl > LK_MAXL || c.nt < 1 || c.nt > LK_MAXT || nblocks < 1 || !n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lock_apply_kernel, dim3(nblocks), dim3(LK_NT), 0, s, c, (const double2*)coef, (double2*)V,
                       (float2*)V32, ld, n);
    return hipGetLastError();
}

hipError_t launch_lock_update(const LockBasis& b, const void* V, const void* V32, void* U, void* U32, size_t ld,
                              size_t n, const void* C, const double* theta, int nblocks, double* npart, double* norms,
                              hipStream_t s) {
    // the kernel holds K <= 3 na basis columns ([X_A W_A P_A])
    if (b.na < 1 || b.na > LK_NA || b.K < b.na || b.K > 3 * b.na || nblocks < 1 || !n) return hipErrorInvalidValue;
    if ((V32 == nullptr) != (U32 == nullptr)) return hipErrorInvalidValue;
    // a basis of K <= 3 na columns: the 4-output instance when na <= 4
    auto kern = b.na <= 4 ? lock_update_kernel<4> : lock_update_kernel<LK_NA>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(LK_NT), 0, s, b, (const double2*)V, (const float2*)V32,
                       (double2*)U, (float2*)U32, ld, n, (const double2*)C, theta, npart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(npart, nblocks, 2 * b.na, norms, s);
}

}  // namespace mfd
