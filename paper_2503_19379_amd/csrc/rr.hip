// Rayleigh-Ritz step of the block eigensolver, on the device, one workgroup.
//
// Section 5.1 takes the eigenpairs from LOBPCG, which minimises the Rayleigh
// quotient over span[X, W, P] at every step.  Given the Gram matrices
// Gs = S^H S and Ga = S^H A S of the basis S = [X, W, P] this kernel returns
// coefficients C with S C = the mb lowest Ritz vectors, and their Ritz values:
//   0. keep the nonzero columns (soft locking has already left converged
//      bands' W and P out of the basis), scale each to unit norm
//      (d = diag(Gs)^-1/2);
//   1. Cholesky factor D Gs D = R^H R column by column; a column whose pivot
//      (squared distance to the span of the previous columns) falls below a
//      threshold is dropped, W and P columns alike;
//   2. Z = R^-1, restricted to the columns kept: Z^H D Gs D Z = I;
//   3. H = Z^H (D Ga D) Z, the operator in that orthonormal basis;
//   4. Householder reduction H = Q T Q^H with T real symmetric tridiagonal
//      (every reflector chosen so that the subdiagonal comes out real);
//      Z <- Z Q;
//   5. the mb lowest eigenvalues of T by bisection on Sturm counts, their
//      eigenvectors by inverse iteration (LU of T - lambda I with partial
//      pivoting), orthogonalised by modified Gram-Schmidt within clusters of
//      close eigenvalues; the Ritz values are the Rayleigh quotients of T;
//   6. C = D Z Y, scattered back to the basis rows.
// The sequential parts (Cholesky, inverse, reduction, bisection, inverse
// iteration) run in one wave with no barrier: the wave's lanes own columns
// (rows) of the small matrices in LDS, and a wave's LDS accesses complete in
// program order.  The dense products use the whole workgroup.
#include "common.h"
#include "solver.h"

namespace mfd {

using C128 = double2;
constexpr int RR_NT = 256;
constexpr int RR_KMAX = 66;
constexpr int RR_MBMAX = 22;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// LDS layout (bytes): A [KMAX][LD] c128 | B [KMAX][LD] c128 | vectors
struct RRShared {
    int idx[RR_KMAX];          // compact index -> basis column
    int vl[RR_KMAX];           // valid (kept and not dropped) compact indices
    double dsc[RR_KMAX];
    int dropped[RR_KMAX];
    double d[RR_KMAX], e[RR_KMAX], lam[RR_KMAX];
    C128 tau[RR_KMAX];
    C128 vv[RR_KMAX], ww[RR_KMAX];
    int cl0[RR_KMAX];          // first member of an eigenvalue's cluster
    int Kk, Kv, dropP;
};

__global__ __launch_bounds__(RR_NT) void rr_kernel(RRArgs a) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ RRShared sh;
    const int mb = a.mb;
    const int K = a.K;
    const int Q2 = 2 * K;
    const int pbeg = mb + a.nw;   // first P column of the basis
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    long long tstamp[6];
    tstamp[0] = wall_clock64();

    // 0. kept columns and their scaling
    if (tid == 0) {
        int kk = 0;
        for (int j = 0; j < K; ++j)
            if (a.G[j * Q2 + j].x > 0.0) sh.idx[kk++] = j;
        sh.Kk = kk;
        sh.dropP = 0;
    }
    __syncthreads();
    const int Kk = sh.Kk;
    const int LD = Kk | 1;   // odd row stride: lanes reading a column hit distinct bank groups
    C128* A = reinterpret_cast<C128*>(smem_raw);   // Kk x LD: Gs -> R -> Z -> Z Q
    C128* B = A + (size_t)Kk * LD;                  // Kk x LD: Ga -> T1 -> H -> reflectors -> workspace
    if (tid < Kk) {
        sh.dropped[tid] = 0;
        sh.dsc[tid] = 1.0 / sqrt(a.G[sh.idx[tid] * Q2 + sh.idx[tid]].x);
    }
    __syncthreads();
    for (int q = tid; q < Kk * Kk; q += RR_NT) {
        const int i = q / Kk, j = q % Kk;
        const int gi = sh.idx[i], gj = sh.idx[j];
        const double s = sh.dsc[i] * sh.dsc[j];
        const C128 gs = a.G[gi * Q2 + gj];
        const C128 g1 = a.G[gi * Q2 + K + gj], g2 = a.G[gj * Q2 + K + gi];
        A[i * LD + j] = mk<C128>(gs.x * s, gs.y * s);
        B[i * LD + j] = mk<C128>(0.5 * (g1.x + g2.x) * s, 0.5 * (g1.y - g2.y) * s);
    }
    __syncthreads();
    tstamp[1] = wall_clock64();

    // 1. Cholesky with column dropping, one wave: lane l owns column l of the
    //    upper factor (rows 0..l of A)
    if (wave == 0) {
        for (int j = 0; j < Kk; ++j) {
            const double piv = A[j * LD + j].x;
            const bool isP = sh.idx[j] >= pbeg;
            const double thr = isP ? a.drop_p : a.drop_w;
            const bool drop = !(piv > thr);
            __builtin_amdgcn_wave_barrier();
            if (drop) {
                if (lane == 0) {
                    sh.dropped[j] = 1;
                    if (isP) sh.dropP = 1;
                }
                for (int l = lane; l < Kk; l += 64)
                    if (l >= j) A[j * LD + l] = mk<C128>(l == j ? 1.0 : 0.0, 0.0);
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            const double rjj = sqrt(piv), inv = 1.0 / rjj;
            for (int l = lane; l < Kk; l += 64) {
                if (l > j) A[j * LD + l] = cscale(A[j * LD + l], inv);
                else if (l == j) A[j * LD + l] = mk<C128>(rjj, 0.0);
            }
            __builtin_amdgcn_wave_barrier();
            // trailing update of the upper triangle: A[i][l] -= conj(R[j][i]) R[j][l], j < i <= l
            for (int l = lane; l < Kk; l += 64) {
                if (l <= j) continue;
                const C128 rl = A[j * LD + l];
                for (int i = j + 1; i <= l; ++i) {
                    const C128 ri = A[j * LD + i];
                    C128 v = A[i * LD + l];
                    v.x -= ri.x * rl.x + ri.y * rl.y;
                    v.y -= ri.x * rl.y - ri.y * rl.x;
                    A[i * LD + l] = v;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // isolate dropped columns: R becomes the identity in their rows and columns
        for (int l = lane; l < Kk; l += 64)
            for (int i = 0; i < Kk; ++i)
                if (i != l && (sh.dropped[i] || sh.dropped[l])) A[i * LD + l] = mk<C128>(0.0, 0.0);
        __builtin_amdgcn_wave_barrier();
        // 2. Z = R^-1 in place (upper), column j from the columns before it:
        //    Z[i][j] = -sum_{i <= l < j} Z[i][l] R[l][j] / R[j][j]; lane i owns row i
        for (int j = 0; j < Kk; ++j) {
            const double inv = 1.0 / A[j * LD + j].x;
            C128 s[2] = {mk<C128>(0.0, 0.0), mk<C128>(0.0, 0.0)};
            for (int h = 0; h < 2; ++h) {
                const int i = lane + 64 * h;
                if (i < j)
                    for (int l = i; l < j; ++l) s[h] = cfma(s[h], A[i * LD + l], A[l * LD + j]);
            }
            __builtin_amdgcn_wave_barrier();
            for (int h = 0; h < 2; ++h) {
                const int i = lane + 64 * h;
                if (i < j) A[i * LD + j] = mk<C128>(-s[h].x * inv, -s[h].y * inv);
            }
            if (lane == 0) A[j * LD + j] = mk<C128>(inv, 0.0);
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) {
            int kv = 0;
            for (int j = 0; j < Kk; ++j)
                if (!sh.dropped[j]) sh.vl[kv++] = j;
            sh.Kv = kv;
        }
    }
    __syncthreads();
    tstamp[2] = wall_clock64();
    const int Kv = sh.Kv;

    // 3. T1 = Bh Zv (Kk x Kv), then Zv = the valid columns of Z packed to the
    //    left of A, then H = Zv^H T1 (Kv x Kv) into B; Z is upper triangular
    constexpr int PER = (RR_KMAX * RR_KMAX + RR_NT - 1) / RR_NT;
    {
        C128 t[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            t[q] = mk<C128>(0.0, 0.0);
            if (e < Kk * Kv) {
                const int i = e / Kv, b = e % Kv, c = sh.vl[b];
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l <= c; ++l) s = cfma(s, B[i * LD + l], A[l * LD + c]);
                t[q] = s;
            }
        }
        C128 z[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            z[q] = mk<C128>(0.0, 0.0);
            if (e < Kk * Kv) {
                const int i = e / Kv, b = e % Kv, c = sh.vl[b];
                if (i <= c) z[q] = A[i * LD + c];   // Z is upper triangular (A keeps Gs below)
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < Kk * Kv) {
                const int i = e / Kv, b = e % Kv;
                B[i * LD + b] = t[q];
                A[i * LD + b] = z[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            t[q] = mk<C128>(0.0, 0.0);
            if (e < Kv * Kv) {
                const int i = e / Kv, j = e % Kv;
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l < Kk; ++l) s = cfmac(s, A[l * LD + i], B[l * LD + j]);
                t[q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < Kv * Kv) B[(e / Kv) * LD + e % Kv] = t[q];
        }
        __syncthreads();
        // Hermitian part
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < Kv * Kv) {
                const int i = e / Kv, j = e % Kv;
                const C128 u = B[i * LD + j], v = B[j * LD + i];
                t[q] = (i == j) ? mk<C128>(u.x, 0.0) : mk<C128>(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < Kv * Kv) B[(e / Kv) * LD + e % Kv] = t[q];
        }
        __syncthreads();
    }
    tstamp[3] = wall_clock64();

    // 4. Householder reduction to real tridiagonal, one wave.  Step j takes
    //    x = H[j+1:, j] and the reflector I - tau v v^H (v[0] = 1) with
    //    (I - tau v v^H)^H x = beta e_1, beta real; then
    //    H22 <- H22 - v w^H - w v^H with p = tau H22 v, w = p - (tau/2)(p^H v) v.
    //    Lane i owns column i of the trailing block (B[l][i] over l); v is kept
    //    in B[l][j], l > j.
    if (wave == 0) {
        for (int j = 0; j + 1 < Kv; ++j) {
            double xn2 = 0.0;
            for (int l = lane; l < Kv; l += 64)
                if (l >= j + 2) xn2 += cabs2(B[l * LD + j]);
            xn2 = wave_sum(xn2);
            const C128 alpha = B[(j + 1) * LD + j];
            double beta;
            C128 t, den;
            if (xn2 == 0.0 && alpha.y == 0.0) {
                t = mk<C128>(0.0, 0.0);
                beta = alpha.x;
                den = mk<C128>(1.0, 0.0);
            } else {
                const double nrm = sqrt(cabs2(alpha) + xn2);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                t = mk<C128>((beta - alpha.x) / beta, -alpha.y / beta);
                den = mk<C128>(alpha.x - beta, alpha.y);   // v = x / (alpha - beta)
            }
            const double dd = cabs2(den);
            const C128 rden = mk<C128>(den.x / dd, -den.y / dd);
            __builtin_amdgcn_wave_barrier();
            for (int l = lane; l < Kv; l += 64) {
                if (l < j + 1) continue;
                const C128 v = (l == j + 1) ? mk<C128>(1.0, 0.0) : cmul(B[l * LD + j], rden);
                B[l * LD + j] = v;
                sh.vv[l] = v;
            }
            if (lane == 0) {
                sh.tau[j] = t;
                sh.e[j] = beta;
                sh.d[j] = B[j * LD + j].x;
            }
            __builtin_amdgcn_wave_barrier();
            if (t.x != 0.0 || t.y != 0.0) {
                // p_i = tau sum_l H[i][l] v_l = tau sum_l conj(H[l][i]) v_l
                C128 p[2] = {mk<C128>(0.0, 0.0), mk<C128>(0.0, 0.0)};
                double hr = 0.0, hi = 0.0;   // p^H v
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    if (i < j + 1 || i >= Kv) continue;
                    C128 s = mk<C128>(0.0, 0.0);
                    for (int l = j + 1; l < Kv; ++l) s = cfmac(s, B[l * LD + i], sh.vv[l]);
                    p[h] = cmul(t, s);
                    const C128 vi = sh.vv[i];
                    hr += p[h].x * vi.x + p[h].y * vi.y;
                    hi += p[h].x * vi.y - p[h].y * vi.x;
                }
                hr = wave_sum(hr);
                hi = wave_sum(hi);
                // alpha2 = -(tau / 2) (p^H v)
                const C128 al = mk<C128>(-0.5 * (t.x * hr - t.y * hi), -0.5 * (t.x * hi + t.y * hr));
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    if (i < j + 1 || i >= Kv) continue;
                    sh.ww[i] = cfma(p[h], al, sh.vv[i]);
                }
                __builtin_amdgcn_wave_barrier();
                for (int h = 0; h < 2; ++h) {
                    const int i = lane + 64 * h;
                    if (i < j + 1 || i >= Kv) continue;
                    const C128 wi = sh.ww[i], vi = sh.vv[i];
                    for (int l = j + 1; l < Kv; ++l) {
                        const C128 vl = sh.vv[l], wl = sh.ww[l];
                        C128 x = B[l * LD + i];
                        // x -= v_l conj(w_i) + w_l conj(v_i)
                        x.x -= vl.x * wi.x + vl.y * wi.y + wl.x * vi.x + wl.y * vi.y;
                        x.y -= vl.y * wi.x - vl.x * wi.y + wl.y * vi.x - wl.x * vi.y;
                        B[l * LD + i] = x;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (lane == 0 && Kv > 0) {
            sh.d[Kv - 1] = B[(Kv - 1) * LD + Kv - 1].x;
            sh.e[Kv - 1] = 0.0;
        }
    }
    __syncthreads();

    // Z <- Z Q = Z H_0 H_1 ... H_{Kv-2}: (Z H)[r][l] = Z[r][l] - tau (Z v)_r conj(v_l).
    // Every wave takes 16 rows of Z, 4 lanes per row splitting l; no barrier.
    {
        const int r = wave * 16 + (lane >> 2), sub = lane & 3;
        const int nrow = Kk;
        for (int j = 0; j + 1 < Kv; ++j) {
            const C128 t = sh.tau[j];
            if (t.x == 0.0 && t.y == 0.0) continue;
            for (int rr = r; rr < nrow; rr += 64) {
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = j + 1 + sub; l < Kv; l += 4) s = cfma(s, A[rr * LD + l], B[l * LD + j]);
                s.x += __shfl_xor(s.x, 1);
                s.y += __shfl_xor(s.y, 1);
                s.x += __shfl_xor(s.x, 2);
                s.y += __shfl_xor(s.y, 2);
                const C128 ts = cmul(t, s);
                for (int l = j + 1 + sub; l < Kv; l += 4) {
                    const C128 v = B[l * LD + j];
                    C128 z = A[rr * LD + l];
                    // z -= ts conj(v)
                    z.x -= ts.x * v.x + ts.y * v.y;
                    z.y -= ts.y * v.x - ts.x * v.y;
                    A[rr * LD + l] = z;
                }
            }
        }
    }
    __syncthreads();
    tstamp[4] = wall_clock64();

    // 5. lowest nsel eigenpairs of T (d, e; Kv x Kv), one wave; B is free now:
    //    per-lane LU workspace and the eigenvectors Y (Kv x nsel, real)
    const int nsel = min(mb, Kv);
    double* Y = reinterpret_cast<double*>(B);                 // [Kv][nsel]
    double* U0 = Y + (size_t)RR_KMAX * RR_MBMAX;               // [Kv][nsel] each
    double* U1 = U0 + (size_t)RR_KMAX * RR_MBMAX;
    double* U2 = U1 + (size_t)RR_KMAX * RR_MBMAX;
    double* ML = U2 + (size_t)RR_KMAX * RR_MBMAX;
    unsigned char* SW = reinterpret_cast<unsigned char*>(ML + (size_t)RR_KMAX * RR_MBMAX);
    if (wave == 0) {
        const int n = Kv;
        // Gershgorin interval and the pivot floor of the Sturm counts
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < n; ++i) {
            const double r = (i ? fabs(sh.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(sh.e[i]) : 0.0);
            lo = fmin(lo, sh.d[i] - r);
            hi = fmax(hi, sh.d[i] + r);
        }
        const double tn = fmax(fabs(lo), fabs(hi));
        const double eps = 2.220446049250313e-16;
        const double pivmin = fmax(2.2250738585072014e-308, eps * eps * tn * 1e-8);
        lo -= 4.0 * eps * tn * n + pivmin;
        hi += 4.0 * eps * tn * n + pivmin;
        // bisection: lane r finds the (r+1)-th smallest eigenvalue
        if (lane < nsel) {
            const int r = lane;
            double x0 = lo, x1 = hi;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (x0 + x1);
                if (!(x1 - x0 > 2.0 * eps * fmax(fabs(x0), fabs(x1)) + pivmin) || mid <= x0 || mid >= x1) break;
                int cnt = 0;
                double q = sh.d[0] - mid;
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += q < 0.0;
                for (int i = 1; i < n; ++i) {
                    const double ei = sh.e[i - 1];
                    q = (sh.d[i] - mid) - ei * ei / q;
                    if (fabs(q) < pivmin) q = -pivmin;
                    cnt += q < 0.0;
                }
                if (cnt > r) x1 = mid;
                else x0 = mid;
            }
            sh.lam[r] = 0.5 * (x0 + x1);
        }
        if (lane == 0) *a.floor = (double)n * eps * tn;
        __builtin_amdgcn_wave_barrier();
        // clusters: consecutive eigenvalues closer than 1e-3 |T|
        const double ortol = 1e-3 * tn;
        if (lane < nsel) {
            int c0 = lane;
            while (c0 > 0 && sh.lam[c0] - sh.lam[c0 - 1] <= ortol) --c0;
            sh.cl0[lane] = c0;
        }
        __builtin_amdgcn_wave_barrier();
        // inverse iteration: (T - lambda_r I) y = b, LU with partial pivoting
        // (lane r), then modified Gram-Schmidt within the cluster (whole wave)
        const double tiny = eps * tn + pivmin;
        for (int it = 0; it < 3; ++it) {
            if (lane < nsel) {
                const int r = lane;
                const double lr = sh.lam[r];
                auto at = [&](double* M, int i) -> double& { return M[(size_t)i * nsel + r]; };
                // right-hand side: a fixed pseudo-random start, then the previous iterate
                double bmax = 0.0;
                for (int i = 0; i < n; ++i) {
                    double b;
                    if (it == 0) {
                        unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(r * 40503u + 12345u);
                        h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
                        b = ((double)(h & 0xffff) + 1.0) / 65536.0 - 0.5;
                    } else {
                        b = at(Y, i);
                    }
                    at(Y, i) = b;
                    bmax = fmax(bmax, fabs(b));
                }
                const double bs = bmax > 0.0 ? 1.0 / bmax : 1.0;
                double p0 = sh.d[0] - lr, p1 = n > 1 ? sh.e[0] : 0.0, p2 = 0.0;
                double bk = at(Y, 0) * bs;
                for (int k = 0; k + 1 < n; ++k) {
                    const double q0 = sh.e[k], q1 = sh.d[k + 1] - lr, q2 = k + 2 < n ? sh.e[k + 1] : 0.0;
                    double bn = at(Y, k + 1) * bs;
                    double m;
                    if (fabs(q0) > fabs(p0)) {
                        at(U0, k) = q0;
                        at(U1, k) = q1;
                        at(U2, k) = q2;
                        SW[(size_t)k * nsel + r] = 1;
                        m = p0 / q0;
                        const double np0 = p1 - m * q1, np1 = p2 - m * q2;
                        p0 = np0; p1 = np1; p2 = 0.0;
                        const double tb = bk; bk = bn; bn = tb;
                    } else {
                        if (p0 == 0.0) p0 = tiny;
                        at(U0, k) = p0;
                        at(U1, k) = p1;
                        at(U2, k) = p2;
                        SW[(size_t)k * nsel + r] = 0;
                        m = q0 / p0;
                        const double np0 = q1 - m * p1, np1 = q2 - m * p2;
                        p0 = np0; p1 = np1; p2 = 0.0;
                    }
                    at(ML, k) = m;
                    at(Y, k) = bk;          // the eliminated right-hand side
                    bk = bn - m * bk;
                }
                if (p0 == 0.0) p0 = tiny;
                at(U0, n - 1) = p0;
                at(Y, n - 1) = bk;
                // back substitution
                double y1 = 0.0, y2 = 0.0, ymax = 0.0;
                for (int k = n - 1; k >= 0; --k) {
                    double s = at(Y, k);
                    if (k + 1 < n) s -= at(U1, k) * y1;
                    if (k + 2 < n) s -= at(U2, k) * y2;
                    double u = at(U0, k);
                    if (fabs(u) < tiny) u = u < 0.0 ? -tiny : tiny;
                    const double y = s / u;
                    at(Y, k) = y;
                    y2 = y1;
                    y1 = y;
                    ymax = fmax(ymax, fabs(y));
                }
                const double ys = ymax > 0.0 && ymax < 1e300 ? 1.0 / ymax : 1.0;
                for (int k = 0; k < n; ++k) at(Y, k) *= ys;
            }
            __builtin_amdgcn_wave_barrier();
            // modified Gram-Schmidt within clusters, then unit length
            for (int r = 0; r < nsel; ++r) {
                const int c0 = sh.cl0[r];
                for (int s2 = c0; s2 < r; ++s2) {
                    double dt = 0.0;
                    for (int i = lane; i < n; i += 64) dt += Y[(size_t)i * nsel + s2] * Y[(size_t)i * nsel + r];
                    dt = wave_sum(dt);
                    for (int i = lane; i < n; i += 64) Y[(size_t)i * nsel + r] -= dt * Y[(size_t)i * nsel + s2];
                    __builtin_amdgcn_wave_barrier();
                }
                double nn = 0.0;
                for (int i = lane; i < n; i += 64) nn += Y[(size_t)i * nsel + r] * Y[(size_t)i * nsel + r];
                nn = wave_sum(nn);
                const double sc = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
                for (int i = lane; i < n; i += 64) Y[(size_t)i * nsel + r] *= sc;
                __builtin_amdgcn_wave_barrier();
            }
        }
        // Ritz values: Rayleigh quotients y^T T y
        if (lane < nsel) {
            const int r = lane;
            double s = 0.0;
            for (int i = 0; i < n; ++i) {
                const double yi = Y[(size_t)i * nsel + r];
                s += sh.d[i] * yi * yi;
                if (i + 1 < n) s += 2.0 * sh.e[i] * yi * Y[(size_t)(i + 1) * nsel + r];
            }
            sh.lam[r] = s;
        }
    }
    __syncthreads();

    // 6. C = D Zv Y (rows idx[j]); columns beyond the kept rank keep their X
    //    column (theta = its Rayleigh quotient) so that X never loses a column
    for (int q = tid; q < K * mb; q += RR_NT) a.C[q] = mk<C128>(0.0, 0.0);
    __syncthreads();
    for (int q = tid; q < Kk * nsel; q += RR_NT) {
        const int j = q / nsel, r = q % nsel;
        C128 s = mk<C128>(0.0, 0.0);
        for (int b = 0; b < Kv; ++b) {
            const double y = Y[(size_t)b * nsel + r];
            const C128 z = A[j * LD + b];
            s.x += z.x * y;
            s.y += z.y * y;
        }
        a.C[sh.idx[j] * mb + r] = mk<C128>(sh.dsc[j] * s.x, sh.dsc[j] * s.y);
    }
    if (tid < nsel) a.theta[tid] = sh.lam[tid];
    for (int r = nsel + tid; r < mb; r += RR_NT) {
        a.C[r * mb + r] = mk<C128>(1.0, 0.0);
        a.theta[r] = a.G[r * Q2 + K + r].x / a.G[r * Q2 + r].x;
    }
    if (tid == 0) {
        a.info[0] = Kv;
        a.info[1] = sh.dropP;
        a.info[2] = a.nw;
        a.info[3] = 0;
        tstamp[5] = wall_clock64();
        for (int q = 0; q < 5; ++q) a.info[4 + q] = (int)(tstamp[q + 1] - tstamp[q]);   // phase ticks
        a.info[9] = Kk;
    }
}

hipError_t launch_rr(const RRArgs& a, hipStream_t s) {
    const int K = a.K;
    if (K > RR_KMAX || K < a.mb || a.mb > RR_MBMAX || a.nw < 0 || a.mb + a.nw > K) return hipErrorInvalidValue;
    const int LD = K | 1;
    const size_t mats = (size_t)2 * K * LD * sizeof(C128);
    // the eigenvector workspace (Y, the LU factors, multipliers and swaps) reuses B
    const size_t work = (size_t)5 * RR_KMAX * RR_MBMAX * sizeof(double) + (size_t)RR_KMAX * RR_MBMAX;
    const size_t lds = std::max(mats, (size_t)K * LD * sizeof(C128) + work);
    hipError_t e = hipFuncSetAttribute((const void*)rr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rr_kernel, dim3(1), dim3(RR_NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace mfd
