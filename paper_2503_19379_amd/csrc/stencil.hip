// Fused application of the compensated MFD operator
//   w = A (M_0 (A' v)) + gamma B' (B v) + c v          (eq. (Ker_comp), Remark 5.1)
// for a block of complex face fields, second-order stencils (Table FD_1D, k = 1).
//
// Per axis i the operators of eqs. (discre), (blocks) are two-point stencils
//   (D_i u)[r]  = u[r+1] cp_i + u[r] cm_i,      cp_i = 1/h + i alpha_i/2, cm_i = -1/h + i alpha_i/2
//   (D_i' u)[r] = u[r-1] conj(cp_i) + u[r] conj(cm_i)
// and A' (eq. (derived_uniform_grid)), A, B, B' are assembled from them as in
// eq. (discrete_2nd_block):
//   e = A'v : e1 = D3'v2 - D2'v3,  e2 = D1'v3 - D3'v1,  e3 = D2'v1 - D1'v2
//   e <- mu e  (M_0, diagonal on edges)
//   w = A e : w1 = D2 e3 - D3 e2,  w2 = D3 e1 - D1 e3,  w3 = D1 e2 - D2 e1
//   q = B v = D1 v1 + D2 v2 + D3 v3,   w_i += gamma D_i' q.
//
// Two kernels, both HBM-bound in intent (v read once, w written once, mu read
// from HBM about once per launch: the bands of a tile run side by side and
// share it in L2): stencil_wave_kernel for N = 64 (below) and, for the other
// grids, stencil_kernel.  In stencil_kernel a workgroup owns an x-y tile of
// N x TY cells plus one halo row on each side in y (x is a full periodic row,
// so x neighbours never leave the tile) and marches through a chunk of z
// planes.  Each thread owns one (x, y)
// column and keeps its z history in registers; in-plane neighbours travel
// through LDS.  Intermediates e = mu A'v and q = Bv never touch HBM.  At step
// t the plane v(t+1) is loaded and the thread forms e(t+1), the in-plane part
// of q(t+1), q(t) (adding the z term from v(t), v(t+1)) and finally w(t) from
// e(t), e(t+1), q(t-1), q(t).
#include "common.h"
#include "internal.h"
#include <algorithm>

namespace mfd {

// R: arithmetic precision; S: storage precision of X and Y (FP32 storage
// with FP64 arithmetic keeps the operator's rounding at the FP64 level).
template <class R, class S = R>
struct StencilArgs {
    const cplx<S>* X;
    cplx<S>* Y;
    const R* mu;          // [3][N][N][N]
    int N, nyt, nzc, zc, nb;
    FieldList fl;
    cplx<R> cp[3], cm[3];
    cplx<R> gcp[3], gcm[3];   // gamma cp, gamma cm
    R gamma, shift;
};

// MAXT: the largest workgroup the instantiation serves (N (TY + 2) threads);
// grids up to N = 64 use at most 640, which leaves each thread more registers.
template <class R, class S, int TY, int MAXT>
__global__ __launch_bounds__(MAXT) void stencil_kernel(StencilArgs<R, S> a) {
    using T = cplx<R>;
    using TS = cplx<S>;
    extern __shared__ unsigned char smem_raw[];
    T* smem = reinterpret_cast<T*>(smem_raw);
    constexpr int ROWS = TY + 2;
    const int N = a.N;
    const int plane_cells = ROWS * N;
    T* vbuf = smem;                      // [3][ROWS][N]
    T* ebuf = smem + 3 * plane_cells;    // [2][3][ROWS][N]
    T* qbuf = smem + 9 * plane_cells;    // [ROWS][N]

    const int tx = threadIdx.x;
    const int ty = threadIdx.y;
    // band fastest, then y tile, then z chunk: the bands of one tile run side
    // by side on one XCD and share its mu planes and halo rows in L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int band = bid % a.nb;
    const int rest = bid / a.nb;
    const int ytile = rest % a.nyt;
    const int zch = rest / a.nyt;

    const int y0 = ytile * TY;
    const int yg = (y0 - 1 + ty + N) % N;
    const int z0 = zch * a.zc;
    const int z1 = z0 + a.zc;
    const size_t NN = (size_t)N * N;
    const size_t N3 = NN * N;
    const TS* Xb = a.X + (size_t)a.fl(band) * 3 * N3;
    TS* Yb = a.Y + (size_t)a.fl(band) * 3 * N3;

    const int txp = (tx + 1 == N) ? 0 : tx + 1;
    const int txm = (tx == 0) ? N - 1 : tx - 1;
    const int row = ty * N;

    const T cp1 = a.cp[0], cp2 = a.cp[1], cp3 = a.cp[2];
    const T cm1 = a.cm[0], cm2 = a.cm[1], cm3 = a.cm[2];
    const R gam = a.gamma, sh = a.shift;

    const T zero = mk<T>(0.0, 0.0);
    T vp0 = zero, vp1 = zero, vp2 = zero;        // v(t) at own cell
    T ec0 = zero, ec1 = zero, ec2 = zero;        // e(t) at own cell
    T qxy_c = zero;                              // in-plane part of q(t)
    T q_prev = zero;                             // q(t-1)

    // v and mu of each plane are loaded two steps ahead, so that their HBM
    // latency overlaps two planes' LDS work and barriers.  Two register sets
    // alternate, A for the planes t + 1 with t - z0 even, B for the odd ones.
    struct Plane {
        TS v0, v1, v2;
        R m0, m1, m2;
    };
    auto load_plane = [&](Plane& P, int t) {   // plane t + 1 (periodic)
        const size_t o = (size_t)((t + 1 + 2 * N) % N) * NN + (size_t)yg * N + tx;
        P.v0 = Xb[o];
        P.v1 = Xb[N3 + o];
        P.v2 = Xb[2 * N3 + o];
        P.m0 = a.mu[o];
        P.m1 = a.mu[N3 + o];
        P.m2 = a.mu[2 * N3 + o];
    };
    auto step = [&](int t, const Plane& P) {
        const TS sv0 = P.v0, sv1 = P.v1, sv2 = P.v2;
        const R mu0 = P.m0, mu1 = P.m1, mu2 = P.m2;
        const T vn0 = mk<T>(sv0.x, sv0.y);
        const T vn1 = mk<T>(sv1.x, sv1.y);
        const T vn2 = mk<T>(sv2.x, sv2.y);
        vbuf[row + tx] = vn0;
        vbuf[plane_cells + row + tx] = vn1;
        vbuf[2 * plane_cells + row + tx] = vn2;
        __syncthreads();

        // e(t+1) = mu A'v at own cell (needs the row below: ty >= 1)
        T en0 = zero, en1 = zero, en2 = zero;
        if (ty >= 1) {
            const T v1ym = vbuf[row - N + tx];
            const T v3ym = vbuf[2 * plane_cells + row - N + tx];
            const T v2xm = vbuf[plane_cells + row + txm];
            const T v3xm = vbuf[2 * plane_cells + row + txm];
            // D3' v2 - D2' v3
            T s = cmulc(cp3, vp1);
            s = cadd(s, cmulc(cm3, vn1));
            s = csub(s, cmulc(cp2, v3ym));
            en0 = csub(s, cmulc(cm2, vn2));
            // D1' v3 - D3' v1
            s = cmulc(cp1, v3xm);
            s = cadd(s, cmulc(cm1, vn2));
            s = csub(s, cmulc(cp3, vp0));
            en1 = csub(s, cmulc(cm3, vn0));
            // D2' v1 - D1' v2
            s = cmulc(cp2, v1ym);
            s = cadd(s, cmulc(cm2, vn0));
            s = csub(s, cmulc(cp1, v2xm));
            en2 = csub(s, cmulc(cm1, vn1));
            en0 = cscale(en0, mu0);
            en1 = cscale(en1, mu1);
            en2 = cscale(en2, mu2);
        }
        // in-plane part of q(t+1) and the full q(t) (needs the row above: ty <= TY)
        T qxy_n = zero, q_t = zero;
        if (ty <= TY) {
            const T v1xp = vbuf[row + txp];
            const T v2yp = vbuf[plane_cells + row + N + tx];
            qxy_n = cmul(cp1, v1xp);
            qxy_n = cfma(qxy_n, cm1, vn0);
            qxy_n = cfma(qxy_n, cp2, v2yp);
            qxy_n = cfma(qxy_n, cm2, vn1);
            q_t = cfma(qxy_c, cp3, vn2);
            q_t = cfma(q_t, cm3, vp2);
        }
        T* eb = ebuf + ((t + 1) & 1) * 3 * plane_cells;
        eb[row + tx] = en0;
        eb[plane_cells + row + tx] = en1;
        eb[2 * plane_cells + row + tx] = en2;
        qbuf[row + tx] = q_t;
        __syncthreads();

        if (t >= z0 && ty >= 1 && ty <= TY) {
            const T* ec = ebuf + (t & 1) * 3 * plane_cells;   // e(t)
            const T e2xp = ec[plane_cells + row + txp];
            const T e3xp = ec[2 * plane_cells + row + txp];
            const T e1yp = ec[row + N + tx];
            const T e3yp = ec[2 * plane_cells + row + N + tx];
            const T qxm = qbuf[row + txm];
            const T qym = qbuf[row - N + tx];
            // w1 = D2 e3 - D3 e2 + gamma D1' q
            T w0 = cmul(cp2, e3yp);
            w0 = cfma(w0, cm2, ec2);
            w0 = csub(w0, cmul(cp3, en1));
            w0 = csub(w0, cmul(cm3, ec1));
            T g0 = cmulc(cp1, qxm);
            g0 = cadd(g0, cmulc(cm1, q_t));
            // w2 = D3 e1 - D1 e3 + gamma D2' q
            T w1 = cmul(cp3, en0);
            w1 = cfma(w1, cm3, ec0);
            w1 = csub(w1, cmul(cp1, e3xp));
            w1 = csub(w1, cmul(cm1, ec2));
            T g1 = cmulc(cp2, qym);
            g1 = cadd(g1, cmulc(cm2, q_t));
            // w3 = D1 e2 - D2 e1 + gamma D3' q
            T w2 = cmul(cp1, e2xp);
            w2 = cfma(w2, cm1, ec1);
            w2 = csub(w2, cmul(cp2, e1yp));
            w2 = csub(w2, cmul(cm2, ec0));
            T g2 = cmulc(cp3, q_prev);
            g2 = cadd(g2, cmulc(cm3, q_t));
            w0 = cadd(w0, cscale(g0, gam));
            w1 = cadd(w1, cscale(g1, gam));
            w2 = cadd(w2, cscale(g2, gam));
            w0 = cadd(w0, cscale(vp0, sh));
            w1 = cadd(w1, cscale(vp1, sh));
            w2 = cadd(w2, cscale(vp2, sh));
            const size_t oo = (size_t)t * NN + (size_t)yg * N + tx;
            Yb[oo] = mk<TS>(w0.x, w0.y);
            Yb[N3 + oo] = mk<TS>(w1.x, w1.y);
            Yb[2 * N3 + oo] = mk<TS>(w2.x, w2.y);
        }
        vp0 = vn0; vp1 = vn1; vp2 = vn2;
        ec0 = en0; ec1 = en1; ec2 = en2;
        qxy_c = qxy_n;
        q_prev = q_t;
    };
    Plane A, B;
    load_plane(A, z0 - 2);
    load_plane(B, z0 - 1);
    for (int t = z0 - 2; t < z1; t += 2) {
        step(t, A);
        load_plane(A, t + 2 < z1 ? t + 2 : t);   // past the chunk: a repeated plane, unused
        if (t + 1 < z1) {                        // uniform: zc + 2 planes, odd for odd zc (N = 100, 120)
            step(t + 1, B);
            load_plane(B, t + 3 < z1 ? t + 3 : t + 1);
        }
    }
}

// Barrier-free form for N = 64: one x row per wave, so x neighbours are
// lanes of the same wave and come through ds_bpermute, and y neighbours are
// registers: each lane owns a strip of WTY rows (plus the halo rows y0 - 1
// and y0 + WTY, whose e and q it recomputes) and marches in z.  No LDS is
// allocated and no wave waits for another, so the memory, FP64 and permute
// work of different waves overlap on a CU.  State carried from plane t to
// t + 1, per lane: v(t) on rows -1..WTY (storage precision), e(t) on rows
// 0..WTY, q(t-1) on rows 0..WTY-1.  At most 168 VGPRs: 3 waves per SIMD.
constexpr int WTY = 2;

__device__ __forceinline__ float lane_get(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(int addr, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class C> __device__ __forceinline__ C lane_get(int addr, C v) {
    v.x = lane_get(addr, v.x);
    v.y = lane_get(addr, v.y);
    return v;
}
// acc - a * b and acc - conj(a) * b, four FMAs each
template <class T> __device__ __forceinline__ T cfms(T acc, T a, T b) {
    acc.x = fma(-a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <class T> __device__ __forceinline__ T cfmsc(T acc, T a, T b) {
    acc.x = fma(-a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

// Grid: a.nyt workgroups of 4 waves (4 consecutive strips) per band and z
// chunk, band next, z chunk slowest; a.nzc chunks of N / nzc planes, rounded.
template <class R, class S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void stencil_wave_kernel(
    StencilArgs<R, S> a) {
    using T = cplx<R>;
    using TS = cplx<S>;
    constexpr int TY = WTY;
    constexpr int N = 64;
    const int x = threadIdx.x & 63;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = bid % a.nyt;
    const int rest = bid / a.nyt;
    const int band = rest % a.nb;
    const int zch = rest / a.nb;
    const int y0 = (grp * 4 + (int)(threadIdx.x >> 6)) * TY;
    const int z0 = zch * N / a.nzc;
    const int z1 = (zch + 1) * N / a.nzc;
    constexpr unsigned NN = N * N;
    constexpr unsigned N3 = NN * N;
    const size_t fo = (size_t)a.fl(band) * 3 * N3;
    const char* Xb = (const char*)(a.X + fo);     // per-lane offsets below stay 32-bit
    char* Yb = (char*)(a.Y + fo);
    const char* Mb = (const char*)a.mu;
    const int am = ((x + N - 1) % N) * 4;         // ds_bpermute address of lane x - 1
    const int ap = ((x + 1) % N) * 4;             // of lane x + 1
    unsigned yo[TY + 2];                          // rows y0 - 1 .. y0 + TY (cell index in a plane)
#pragma unroll
    for (int r = 0; r < TY + 2; ++r) yo[r] = (unsigned)(((y0 - 1 + r + N) % N) * N + x);

    const T cp1 = a.cp[0], cp2 = a.cp[1], cp3 = a.cp[2];
    const T cm1 = a.cm[0], cm2 = a.cm[1], cm3 = a.cm[2];
    const T gp1 = a.gcp[0], gp2 = a.gcp[1], gp3 = a.gcp[2];   // gamma cp, gamma cm
    const T gm1 = a.gcm[0], gm2 = a.gcm[1], gm3 = a.gcm[2];
    const R sh = a.shift;
    auto up = [](TS s) { return mk<T>(s.x, s.y); };

    struct Plane {
        TS v[TY + 2][3];   // rows -1..TY
        R m[TY + 1][3];    // rows 0..TY
    };
    auto load = [&](Plane& P, int z) {            // plane z, -1 <= z <= N
        const unsigned zo = (unsigned)((z + N) % N) * NN;
#pragma unroll
        for (int r = 0; r < TY + 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                P.v[r][c] = *(const TS*)(Xb + (size_t)((c * N3 + zo + yo[r]) * (unsigned)sizeof(TS)));
#pragma unroll
        for (int r = 0; r < TY + 1; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                P.m[r][c] = *(const R*)(Mb + (size_t)((c * N3 + zo + yo[r + 1]) * (unsigned)sizeof(R)));
    };

    struct Vec3 {
        T c[3];
    };
    TS vc[TY + 2][3];   // v(t)
    Vec3 ec[TY + 1];    // e(t) = mu A'v(t)
    T qp[TY];           // q(t-1) = B v(t-1)

    auto e_row = [&](const Plane& P, int r) {     // e(t+1) on row r, 0 <= r <= TY
        const T v0 = up(P.v[r + 1][0]), v1 = up(P.v[r + 1][1]), v2 = up(P.v[r + 1][2]);
        const T v1ym = up(P.v[r][0]), v3ym = up(P.v[r][2]);
        const T v2xm = lane_get(am, v1);
        const T v3xm = lane_get(am, v2);
        const T p0 = up(vc[r + 1][0]), p1 = up(vc[r + 1][1]);
        Vec3 en;
        // D3' v2 - D2' v3
        T s = cmulc(cp3, p1);
        s = cfmac(s, cm3, v1);
        s = cfmsc(s, cp2, v3ym);
        s = cfmsc(s, cm2, v2);
        en.c[0] = cscale(s, P.m[r][0]);
        // D1' v3 - D3' v1
        s = cmulc(cp1, v3xm);
        s = cfmac(s, cm1, v2);
        s = cfmsc(s, cp3, p0);
        s = cfmsc(s, cm3, v0);
        en.c[1] = cscale(s, P.m[r][1]);
        // D2' v1 - D1' v2
        s = cmulc(cp2, v1ym);
        s = cfmac(s, cm2, v0);
        s = cfmsc(s, cp1, v2xm);
        s = cfmsc(s, cm1, v1);
        en.c[2] = cscale(s, P.m[r][2]);
        return en;
    };
    auto q_row = [&](const Plane& P, int r) {     // q(t) on row r, -1 <= r < TY
        const T c0 = up(vc[r + 1][0]), c1 = up(vc[r + 1][1]), c2 = up(vc[r + 1][2]);
        const T c0xp = lane_get(ap, c0);
        const T c1yp = up(vc[r + 2][1]);
        const T n2 = up(P.v[r + 1][2]);
        T s = cmul(cp1, c0xp);
        s = cfma(s, cm1, c0);
        s = cfma(s, cp2, c1yp);
        s = cfma(s, cm2, c1);
        s = cfma(s, cp3, n2);
        return cfma(s, cm3, c2);
    };
    // One plane step: v(t+1) arrives in P; forms e(t+1), q(t) and, when
    // `out`, writes w(t).  Rows are swept upwards and each row's state is
    // replaced as soon as the rows below and above no longer need it:
    // after row r, ec[r] holds e(t+1), qp[r] holds q(t) (the y - 1 term of
    // row r + 1) and vc row r holds v(t+1).
    auto step = [&](int t, const Plane& P, bool out) {
        T qym = q_row(P, -1);
#pragma unroll
        for (int c = 0; c < 3; ++c) vc[0][c] = P.v[0][c];
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const Vec3 en = e_row(P, r);
            const T qc = q_row(P, r);
            if (out) {                            // w(t) on row r
                const T qxm = lane_get(am, qc);
                const T e2xp = lane_get(ap, ec[r].c[1]);
                const T e3xp = lane_get(ap, ec[r].c[2]);
                // w1 = D2 e3 - D3 e2 + gamma D1' q
                T w0 = cmul(cp2, ec[r + 1].c[2]);
                w0 = cfma(w0, cm2, ec[r].c[2]);
                w0 = cfms(w0, cp3, en.c[1]);
                w0 = cfms(w0, cm3, ec[r].c[1]);
                w0 = cfmac(w0, gp1, qxm);
                w0 = cfmac(w0, gm1, qc);
                // w2 = D3 e1 - D1 e3 + gamma D2' q
                T w1 = cmul(cp3, en.c[0]);
                w1 = cfma(w1, cm3, ec[r].c[0]);
                w1 = cfms(w1, cp1, e3xp);
                w1 = cfms(w1, cm1, ec[r].c[2]);
                w1 = cfmac(w1, gp2, qym);
                w1 = cfmac(w1, gm2, qc);
                // w3 = D1 e2 - D2 e1 + gamma D3' q
                T w2 = cmul(cp1, e2xp);
                w2 = cfma(w2, cm1, ec[r].c[1]);
                w2 = cfms(w2, cp2, ec[r + 1].c[0]);
                w2 = cfms(w2, cm2, ec[r].c[0]);
                w2 = cfmac(w2, gp3, qp[r]);
                w2 = cfmac(w2, gm3, qc);
                if (sh != R(0)) {                 // uniform
                    w0 = cadd(w0, cscale(up(vc[r + 1][0]), sh));
                    w1 = cadd(w1, cscale(up(vc[r + 1][1]), sh));
                    w2 = cadd(w2, cscale(up(vc[r + 1][2]), sh));
                }
                const unsigned o = (unsigned)t * NN + yo[r + 1];
                *(TS*)(Yb + (size_t)(o * (unsigned)sizeof(TS))) = mk<TS>(w0.x, w0.y);
                *(TS*)(Yb + (size_t)((N3 + o) * (unsigned)sizeof(TS))) = mk<TS>(w1.x, w1.y);
                *(TS*)(Yb + (size_t)((2 * N3 + o) * (unsigned)sizeof(TS))) = mk<TS>(w2.x, w2.y);
            }
            ec[r] = en;
            qp[r] = qc;
            qym = qc;
#pragma unroll
            for (int c = 0; c < 3; ++c) vc[r + 1][c] = P.v[r + 1][c];
        }
        ec[TY] = e_row(P, TY);
#pragma unroll
        for (int c = 0; c < 3; ++c) vc[TY + 1][c] = P.v[TY + 1][c];
    };

    Plane P;
    load(P, z0 - 1);
#pragma unroll
    for (int r = 0; r < TY + 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) vc[r][c] = P.v[r][c];
    load(P, z0);
    step(z0 - 1, P, false);                       // e(z0), q(z0 - 1)
    for (int t = z0; t < z1; ++t) {
        load(P, t + 1);                           // t + 1 <= N: periodic
        step(t, P, true);
    }
}

// Tile height TY for grid size N: N * (TY + 2) <= 1024 threads, TY | N.
static int stencil_ty(int N) {
    int best = 0;
    for (int ty : {8, 6, 4, 2, 1})
        if (N % ty == 0 && N * (ty + 2) <= 1024) { best = ty; break; }
    return best;
}

template <class R, class S, int TY>
static hipError_t launch_ty(const StencilArgs<R, S>& a, hipStream_t s) {
    const size_t lds = (size_t)10 * (TY + 2) * a.N * sizeof(cplx<R>);
    auto kern = a.N * (TY + 2) <= 640 ? stencil_kernel<R, S, TY, 640> : stencil_kernel<R, S, TY, 1024>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 block(a.N, TY + 2);
    dim3 grid(a.nyt * a.nzc * a.nb);
    hipLaunchKernelGGL(kern, grid, block, lds, s, a);
    return hipGetLastError();
}

template <class R, class S>
static hipError_t launch_wave(StencilArgs<R, S> a, int target, hipStream_t s) {
    constexpr int N = 64, wpc = N * N / (64 * WTY);   // waves per band and z chunk
    a.nyt = wpc / 4;
    // z chunks (of at least 8 planes; each re-reads two halo planes) until
    // the grid has `target` waves
    const size_t per = (size_t)wpc * a.nb;
    a.nzc = (int)std::min<size_t>(std::max<size_t>((target + per - 1) / per, 1), (size_t)N / 8);
    a.zc = 0;
    dim3 grid(a.nyt * a.nb * a.nzc);
    hipLaunchKernelGGL((stencil_wave_kernel<R, S>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class R, class S>
hipError_t launch_stencil_rs(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                             const FieldList& fl) {
    if (fl.on && nb > 32) return hipErrorInvalidValue;
    if (two_pass(p)) return launch_wide<R, S>(p, nb, X, Y, mu, s, fl);
    StencilArgs<R, S> a;
    a.fl = fl;
    a.X = (const cplx<S>*)X;
    a.Y = (cplx<S>*)Y;
    a.mu = (const R*)mu;
    a.N = p.N;
    a.nb = nb;
    const int TY = stencil_ty(p.N);
    if (TY == 0) return hipErrorInvalidValue;
    a.nyt = p.N / TY;
    // z chunks: enough workgroups to fill 256 CUs several times over, chunks
    // of at least 8 planes (each chunk re-reads two halo planes).
    int zc = p.N;
    while (zc % 2 == 0 && zc >= 16 && (size_t)a.nyt * (p.N / zc) * nb < (size_t)p.stencil_wgs) zc /= 2;
    a.zc = zc;
    a.nzc = p.N / zc;
    for (int i = 0; i < 3; ++i) {
        a.cp[i] = mk<cplx<R>>(1.0 / p.h, 0.5 * p.k[i]);
        a.cm[i] = mk<cplx<R>>(-1.0 / p.h, 0.5 * p.k[i]);
        a.gcp[i] = mk<cplx<R>>(p.gamma / p.h, 0.5 * p.gamma * p.k[i]);
        a.gcm[i] = mk<cplx<R>>(-p.gamma / p.h, 0.5 * p.gamma * p.k[i]);
    }
    a.gamma = (R)p.gamma;
    a.shift = (R)p.shift;
    if (p.N == 64) return launch_wave<R, S>(a, p.stencil_wgs, s);
    switch (TY) {
        case 8: return launch_ty<R, S, 8>(a, s);
        case 6: return launch_ty<R, S, 6>(a, s);
        case 4: return launch_ty<R, S, 4>(a, s);
        case 2: return launch_ty<R, S, 2>(a, s);
        default: return launch_ty<R, S, 1>(a, s);
    }
}

template <class R>
hipError_t launch_stencil(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                          const FieldList& fl) {
    return launch_stencil_rs<R, R>(p, nb, X, Y, mu, s, fl);
}

hipError_t launch_stencil_f64_s32(const OpParams& p, int nb, const void* X, void* Y, const void* mu64,
                                  hipStream_t s, const FieldList& fl) {
    return launch_stencil_rs<double, float>(p, nb, X, Y, mu64, s, fl);
}

template hipError_t launch_stencil<float>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                          const FieldList&);
template hipError_t launch_stencil<double>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                           const FieldList&);

}  // namespace mfd
