// Rayleigh-Ritz step by cyclic Jacobi (one workgroup), the accurate route of
// the last iterations of a band solve.
//
// The same step as rr.hip (kept columns, scaled Cholesky with column
// dropping, Z = R^-1, H = Z^H Ga Z), with the eigenproblem of H solved by
// one-phase round-robin cyclic Jacobi: every index is in one pair per round,
// the two-sided update J^H H J one 2 x 2 block per thread (plus Z <- Z J),
// two barriers per round, until the off-diagonal part falls below 1e-12 of
// the diagonal.  Jacobi's eigenvalues and vectors carry errors relative to
// the entries they rotate, so the Ritz values of the wanted (smallest)
// eigenpairs stay accurate beside the stiff directions of the basis, where a
// Householder reduction's accuracy is absolute (eps |H|).  Dropped columns
// (and a padding column when the size is odd) are isolated in H with a huge
// diagonal entry, so they are never selected.
#include "common.h"
#include "solver.h"

namespace mfd {
namespace {

using C128 = double2;
constexpr int RR_NT = 512;
constexpr int RR_KMAX = 66;
constexpr double RR_BIG = 1e300;

struct Rot {
    double c, s;
    C128 em;   // e^{-i phi}
    int p, q;
};

__global__ __launch_bounds__(RR_NT) void rr_jacobi_kernel(RRArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int mb = a.mb;
    const int K = a.K;
    const int Q = 2 * K;
    const int pbeg = mb + a.nw;           // first P column of the basis
    __shared__ int idx[RR_KMAX];        // compact index -> basis column
    __shared__ double dsc[RR_KMAX];
    __shared__ int dropped[RR_KMAX];
    __shared__ double piv_s;
    __shared__ int dropP, Kk_s, active_s;
    __shared__ Rot rot[RR_KMAX / 2];
    __shared__ double redv[2][RR_NT / 64];
    __shared__ int perm[RR_KMAX];
    const int tid = threadIdx.x;
    long long tstamp[6];
    tstamp[0] = wall_clock64();

    // 1. kept columns: the basis holds only the W and P columns of unconverged
    //    bands (soft locking is done by the caller); zero columns are left out
    if (tid == 0) {
        int kk = 0;
        for (int j = 0; j < K; ++j)
            if (a.G[j * Q + j].x > 0.0) idx[kk++] = j;
        Kk_s = kk;
        active_s = a.nw;
        dropP = 0;
    }
    __syncthreads();
    const int Kk = Kk_s;
    const int KE = Kk + (Kk & 1);                  // even size for the pairing
    C128* A = reinterpret_cast<C128*>(smem_raw);   // KE x KE: Gs -> R -> Z
    C128* B = A + KE * KE;                         // KE x KE: Ga -> T -> H
    if (tid < KE) {
        dropped[tid] = (tid >= Kk);
        dsc[tid] = (tid < Kk) ? 1.0 / sqrt(a.G[idx[tid] * Q + idx[tid]].x) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < KE * KE; e += RR_NT) {
        const int i = e / KE, j = e % KE;
        if (i < Kk && j < Kk) {
            const int gi = idx[i], gj = idx[j];
            const double s = dsc[i] * dsc[j];
            const C128 gs = a.G[gi * Q + gj];
            const C128 g1 = a.G[gi * Q + K + gj], g2 = a.G[gj * Q + K + gi];
            A[e] = mk<C128>(gs.x * s, gs.y * s);
            B[e] = mk<C128>(0.5 * (g1.x + g2.x) * s, 0.5 * (g1.y - g2.y) * s);
        } else {
            A[e] = mk<C128>(i == j ? 1.0 : 0.0, 0.0);
            B[e] = mk<C128>(0.0, 0.0);
        }
    }
    __syncthreads();

    tstamp[1] = wall_clock64();
    // 2. Cholesky with column dropping (upper factor R in A)
    for (int j = 0; j < Kk; ++j) {
        if (tid == 0) {
            double rjj = 0.0;
            const bool isP = idx[j] >= pbeg;
            const double piv = A[j * KE + j].x;
            const double thr = isP ? a.drop_p : a.drop_w;
            if (!(piv > thr)) {
                dropped[j] = 1;
                if (isP) dropP = 1;
            } else {
                rjj = sqrt(piv);
            }
            piv_s = rjj;
        }
        __syncthreads();
        const double rjj = piv_s;
        if (rjj > 0.0) {
            const double inv = 1.0 / rjj;
            for (int l = j + 1 + tid; l < Kk; l += RR_NT) A[j * KE + l] = cscale(A[j * KE + l], inv);
            if (tid == 0) A[j * KE + j] = mk<C128>(rjj, 0.0);
            __syncthreads();
            const int m = Kk - j - 1;
            for (int e = tid; e < m * m; e += RR_NT) {
                const int i = j + 1 + e / m, l = j + 1 + e % m;
                if (l >= i) {
                    const C128 ri = A[j * KE + i], rl = A[j * KE + l];
                    C128 v = A[i * KE + l];
                    v.x -= ri.x * rl.x + ri.y * rl.y;
                    v.y -= ri.x * rl.y - ri.y * rl.x;
                    A[i * KE + l] = v;
                }
            }
        }
        __syncthreads();
    }
    // isolate dropped columns
    for (int e = tid; e < KE * KE; e += RR_NT) {
        const int i = e / KE, l = e % KE;
        if (l < i) A[e] = mk<C128>(0.0, 0.0);
        else if (dropped[i] || dropped[l]) A[e] = mk<C128>(i == l ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    tstamp[2] = wall_clock64();
    // 3a. Z = R^-1 in place, column by column (Z[i][j] = -sum_{i<=l<j} Z[i][l] R[l][j] / R[j][j]);
    //     8 threads share each dot product
    for (int j = 0; j < KE; ++j) {
        const double inv = 1.0 / A[j * KE + j].x;
        const int i = tid >> 3, g = tid & 7;
        C128 s = mk<C128>(0.0, 0.0);
        if (i < j)
            for (int l = i + g; l < j; l += 8) s = cfma(s, A[i * KE + l], A[l * KE + j]);
        for (int o = 4; o > 0; o >>= 1) {
            s.x += __shfl_xor(s.x, o, 8);
            s.y += __shfl_xor(s.y, o, 8);
        }
        __syncthreads();
        if (i < j && g == 0) A[i * KE + j] = mk<C128>(-s.x * inv, -s.y * inv);
        if (tid == 0) A[j * KE + j] = mk<C128>(inv, 0.0);
        __syncthreads();
    }
    // 3b. T = Ga Z, then H = Z^H T (register-staged in place in B)
    constexpr int PER = (RR_KMAX * RR_KMAX + RR_NT - 1) / RR_NT;
    {
        C128 t[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            t[q] = mk<C128>(0.0, 0.0);
            if (e < KE * KE) {
                const int i = e / KE, j = e % KE;
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l <= j; ++l) s = cfma(s, B[i * KE + l], A[l * KE + j]);
                t[q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) B[e] = t[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) {
                const int i = e / KE, j = e % KE;
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l <= i; ++l) s = cfmac(s, A[l * KE + i], B[l * KE + j]);
                t[q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) {
                const int i = e / KE, j = e % KE;
                if (dropped[i] || dropped[j]) t[q] = mk<C128>(i == j ? RR_BIG : 0.0, 0.0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) B[e] = t[q];
        }
        __syncthreads();
        // Hermitian part
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) {
                const int i = e / KE, j = e % KE;
                const C128 u = B[e], v = B[j * KE + i];
                t[q] = (i == j) ? mk<C128>(u.x, 0.0) : mk<C128>(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < KE * KE) B[e] = t[q];
        }
        __syncthreads();
    }

    tstamp[3] = wall_clock64();
    // 4. cyclic Jacobi, round-robin pairs, one-phase two-sided rounds
    const int npairs = KE / 2;
    int sweep = 0;
    for (; sweep < 30; ++sweep) {
        double off = 0.0, dn = 0.0;
        for (int e = tid; e < KE * KE; e += RR_NT) {
            const int i = e / KE, j = e % KE;
            if (dropped[i] || dropped[j]) continue;
            const C128 v = B[e];
            if (i == j) dn += v.x * v.x;
            else off += cabs2(v);
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_down(off, o);
            dn += __shfl_down(dn, o);
        }
        if ((tid & 63) == 0) { redv[0][tid >> 6] = off; redv[1][tid >> 6] = dn; }
        __syncthreads();
        off = 0.0; dn = 0.0;
        for (int w = 0; w < RR_NT / 64; ++w) { off += redv[0][w]; dn += redv[1][w]; }
        __syncthreads();
        // off-diagonal at 1e-12 of the diagonal: the Ritz values are then
        // exact to about 1e-24 relative and the vectors to 1e-12 over the
        // relative gap, far inside the 1e-8 residuals the solve works to
        if (off <= 1e-24 * dn || KE <= 1) break;
        for (int r = 0; r < KE - 1; ++r) {
            if (tid < npairs) {
                const int i = tid;
                int p, q;
                if (i == 0) { p = KE - 1; q = r; }
                else { p = (r + i) % (KE - 1); q = (r - i + (KE - 1)) % (KE - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                Rot ro;
                ro.p = p; ro.q = q; ro.c = 1.0; ro.s = 0.0; ro.em = mk<C128>(1.0, 0.0);
                if (!dropped[p] && !dropped[q]) {
                    const C128 b = B[p * KE + q];
                    const double beta = sqrt(cabs2(b));
                    const double ap = B[p * KE + p].x, dq = B[q * KE + q].x;
                    if (beta > 1e-300 && beta > 1e-18 * sqrt(fabs(ap * dq))) {
                        const double tau = (dq - ap) / (2.0 * beta);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        ro.c = 1.0 / sqrt(1.0 + t * t);
                        ro.s = t * ro.c;
                        ro.em = mk<C128>(b.x / beta, -b.y / beta);
                    }
                }
                rot[i] = ro;
            }
            __syncthreads();
            // (a) 2 x 2 blocks of H: rows of pair u, columns of pair v: J_u^H H J_v
            // (b) rows of Z: columns of pair v: Z J_v
            const int nh = npairs * npairs;
            for (int e = tid; e < nh + npairs * KE; e += RR_NT) {
                if (e < nh) {
                    const Rot ru = rot[e / npairs], rv = rot[e % npairs];
                    if (ru.s == 0.0 && rv.s == 0.0) continue;
                    const C128 hpp = B[ru.p * KE + rv.p], hpq = B[ru.p * KE + rv.q];
                    const C128 hqp = B[ru.q * KE + rv.p], hqq = B[ru.q * KE + rv.q];
                    // M = J_u^H H: row p = c h_p - s e^{i phi} h_q, row q = s h_p + c e^{i phi} h_q
                    const C128 eu = mk<C128>(ru.em.x, -ru.em.y);
                    const C128 tq0 = cmul(eu, hqp), tq1 = cmul(eu, hqq);
                    const C128 m00 = mk<C128>(ru.c * hpp.x - ru.s * tq0.x, ru.c * hpp.y - ru.s * tq0.y);
                    const C128 m01 = mk<C128>(ru.c * hpq.x - ru.s * tq1.x, ru.c * hpq.y - ru.s * tq1.y);
                    const C128 m10 = mk<C128>(ru.s * hpp.x + ru.c * tq0.x, ru.s * hpp.y + ru.c * tq0.y);
                    const C128 m11 = mk<C128>(ru.s * hpq.x + ru.c * tq1.x, ru.s * hpq.y + ru.c * tq1.y);
                    // N = M J_v: col p = c m_p - s e^{-i phi} m_q, col q = s m_p + c e^{-i phi} m_q
                    const C128 u0 = cmul(rv.em, m01), u1 = cmul(rv.em, m11);
                    C128 n00 = mk<C128>(rv.c * m00.x - rv.s * u0.x, rv.c * m00.y - rv.s * u0.y);
                    C128 n01 = mk<C128>(rv.s * m00.x + rv.c * u0.x, rv.s * m00.y + rv.c * u0.y);
                    C128 n10 = mk<C128>(rv.c * m10.x - rv.s * u1.x, rv.c * m10.y - rv.s * u1.y);
                    C128 n11 = mk<C128>(rv.s * m10.x + rv.c * u1.x, rv.s * m10.y + rv.c * u1.y);
                    if (ru.p == rv.p) {   // the block of the pair itself: diagonal after the rotation
                        n01 = mk<C128>(0.0, 0.0);
                        n10 = mk<C128>(0.0, 0.0);
                        n00.y = 0.0;
                        n11.y = 0.0;
                    }
                    B[ru.p * KE + rv.p] = n00;
                    B[ru.p * KE + rv.q] = n01;
                    B[ru.q * KE + rv.p] = n10;
                    B[ru.q * KE + rv.q] = n11;
                } else {
                    // consecutive threads take consecutive pairs of one row (unit-stride LDS)
                    const int f = e - nh;
                    const Rot rv = rot[f % npairs];
                    if (rv.s == 0.0) continue;
                    const int row = f / npairs;
                    const C128 zp = A[row * KE + rv.p], zq = A[row * KE + rv.q];
                    const C128 t = cmul(rv.em, zq);
                    A[row * KE + rv.p] = mk<C128>(rv.c * zp.x - rv.s * t.x, rv.c * zp.y - rv.s * t.y);
                    A[row * KE + rv.q] = mk<C128>(rv.s * zp.x + rv.c * t.x, rv.s * zp.y + rv.c * t.y);
                }
            }
            __syncthreads();
        }
    }
    tstamp[4] = wall_clock64();
    // 5. order the eigenvalues, emit coefficients of the lowest mb
    if (tid < KE) {
        const double ti = B[tid * KE + tid].x;
        int rank = 0;
        for (int j = 0; j < KE; ++j) {
            const double tj = B[j * KE + j].x;
            rank += (tj < ti) || (tj == ti && j < tid);
        }
        perm[rank] = tid;
    }
    __syncthreads();
    for (int e = tid; e < K * mb; e += RR_NT) a.C[e] = mk<C128>(0.0, 0.0);
    __syncthreads();
    for (int e = tid; e < Kk * mb; e += RR_NT) {
        const int j = e / mb, r = e % mb;
        const int c = perm[r];
        const C128 z = A[j * KE + c];
        a.C[idx[j] * mb + r] = mk<C128>(dsc[j] * z.x, dsc[j] * z.y);
    }
    if (tid < mb) a.theta[tid] = B[perm[tid] * KE + perm[tid]].x;
    if (tid == 0) {
        double tn = 0.0;
        for (int q = 0; q < Kk; ++q)
            if (!dropped[q]) tn = fmax(tn, fabs(B[q * KE + q].x));
        *a.floor = (double)Kk * 2.220446049250313e-16 * tn;
    }
    if (tid == 0) {
        int nk = 0;
        for (int j = 0; j < Kk; ++j) nk += !dropped[j];
        a.info[0] = nk;
        a.info[1] = dropP;
        a.info[2] = active_s;
        a.info[3] = sweep;
        tstamp[5] = wall_clock64();
        for (int q = 0; q < 5; ++q) a.info[4 + q] = (int)(tstamp[q + 1] - tstamp[q]);   // phase ticks
        a.info[9] = Kk;
    }
}

}  // namespace

hipError_t launch_rr_jacobi(const RRArgs& a, hipStream_t s) {
    const int K = a.K;
    if (K > RR_KMAX || K < a.mb || a.nw < 0 || a.mb + a.nw > K) return hipErrorInvalidValue;
    const int KE = K + (K & 1);
    const size_t lds = (size_t)2 * KE * KE * sizeof(C128);
    hipError_t e = hipFuncSetAttribute((const void*)rr_jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rr_jacobi_kernel, dim3(1), dim3(RR_NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace mfd
