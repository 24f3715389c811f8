// Fused single-pass operator on a general lattice, order 2 (Section 4.2,
// eq. (unified_mat); Section 4.4, eq. (Ker_comp)):
//   w = A M_0 A' v + gamma B'B v + c v,
// with every derivative D^_i = sum_j B_ij K_j + i alpha_i L_i mixing the
// unit-step differences of all three grid axes (B_ij = N (A^-1)_ji) and L_i
// averaging along grid axis i.  For one cell r:
//   (D^_i u)(r)  = sum_j B_ij (u(r + e_j) - u(r)) + i (alpha_i / 2) (u(r + e_i) + u(r)),
//   (D^_i' u)(r) = sum_j B_ij (u(r - e_j) - u(r)) - i (alpha_i / 2) (u(r - e_i) + u(r)),
//   e = M_0 A'v needs v at r and r - e_j;  q = B v needs v at r and r + e_j;
//   w(r) needs e at r and r + e_j, q at r and r - e_j.
// One workgroup owns a 16 x 10 tile of (x, y) for one band and marches up a
// chunk of z.  Per plane it loads v(z + 1) with a one-cell halo into LDS,
// forms e(z + 1) on the tile and one cell beyond on the +x and +y sides,
// q(z) on the tile and one cell before on the -x and -y sides, then w(z).
// Two LDS slots per quantity roll with z, so v is read from HBM once per
// plane (plus the halo ring) and nothing but w is written.
#include "common.h"
#include "internal.h"

namespace mfd {

namespace {

// 16 x 10 tiles: the e and q regions (17 x 11 = 187 entries) take one pass
// of the 256 threads each, w uses 160 of them, and 34.4 KB of LDS (FP32
// storage) lets 4 workgroups share a CU (16 x 14: 3, 16 x 8: 5 were slower)
constexpr int LT_X = 16, LT_Y = 10, LT_NT = 256;
constexpr int LV_X = LT_X + 2, LV_Y = LT_Y + 2;   // v tile with a one-cell halo
constexpr int LE_X = LT_X + 1, LE_Y = LT_Y + 1;   // e: tile + one cell beyond; q: one cell before

template <class R>
struct LatArgs {
    const void* X;
    void* Y;
    const R* mu;
    int N, nb, ntx, nty, nzc;
    R B[3][3];     // B[i][j]: weight of the unit-step difference along grid axis j in D^_i
    R ha[3];       // alpha_i / 2
    R gamma, shift;
    FieldList fl;
};

// i h z
template <class C, class R>
__device__ __forceinline__ C imul(C z, R h) {
    return mk<C>(-h * z.y, h * z.x);
}

template <class R, class S>
__global__ __launch_bounds__(LT_NT) void lattice_fused_kernel(LatArgs<R> a) {
    using C = cplx<R>;
    using CS = cplx<S>;
    extern __shared__ unsigned char smem_raw[];
    C* Es = reinterpret_cast<C*>(smem_raw);                 // [2][3][LE_Y][LE_X]
    C* Qs = Es + 2 * 3 * LE_Y * LE_X;                        // [2][LE_Y][LE_X]
    CS* Vs = reinterpret_cast<CS*>(Qs + 2 * LE_Y * LE_X);    // [2][3][LV_Y][LV_X]
    auto V = [&](int s, int c, int ly, int lx) {
        const CS v = Vs[((s * 3 + c) * LV_Y + ly) * LV_X + lx];
        return mk<C>(v.x, v.y);
    };
    auto E = [&](int s, int c, int ey, int ex) -> C& { return Es[((s * 3 + c) * LE_Y + ey) * LE_X + ex]; };
    auto Q = [&](int s, int qy, int qx) -> C& { return Qs[(s * LE_Y + qy) * LE_X + qx]; };

    const int N = a.N;
    const size_t N3 = (size_t)N * N * N;
    // band fastest, then x tile, y tile, z chunk, and runs of consecutive
    // blocks on one XCD: the bands of a tile share its mu planes, and
    // neighbouring tiles their halo lines, in that XCD's L2
    int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int b = bid % a.nb;
    bid /= a.nb;
    const int tx = bid % a.ntx;
    bid /= a.ntx;
    const int ty = bid % a.nty;
    const int zc = bid / a.nty;
    const int x0 = tx * LT_X, y0 = ty * LT_Y;
    const int z0 = zc * N / a.nzc, z1 = (zc + 1) * N / a.nzc;
    const size_t f = (size_t)a.fl(b) * 3 * N3;
    const CS* X = (const CS*)a.X + f;
    CS* Y = (CS*)a.Y + f;
    const int t = threadIdx.x;
    auto wr = [N](int c) {   // periodic index; c >= -1 here
        c %= N;
        return c < 0 ? c + N : c;
    };

    // v of plane z on the tile and its halo ring into V slot s
    auto fill = [&](int s, int z) {
        for (int i = t; i < LV_X * LV_Y; i += LT_NT) {
            const int lx = i % LV_X, ly = i / LV_X;
            const size_t o = ((size_t)z * N + wr(y0 + ly - 1)) * N + wr(x0 + lx - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) Vs[((s * 3 + c) * LV_Y + ly) * LV_X + lx] = X[c * N3 + o];
        }
    };
    // e(ze) = M_0 A'v into E slot se, from v(ze) (V slot sv) and v(ze - 1) (V slot sb)
    auto make_e = [&](int se, int sv, int sb, int ze) {
        for (int i = t; i < LE_X * LE_Y; i += LT_NT) {
            const int ex = i % LE_X, ey = i / LE_X, lx = ex + 1, ly = ey + 1;
            C dp[3][3];   // dp[c][k] = D^_k' v_c
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const C u = V(sv, c, ly, lx);
                const C ub[3] = {V(sv, c, ly, lx - 1), V(sv, c, ly - 1, lx), V(sb, c, ly, lx)};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    C r = imul(cadd(ub[k], u), -a.ha[k]);
#pragma unroll
                    for (int j = 0; j < 3; ++j) r = cadd(r, cscale(csub(ub[j], u), a.B[k][j]));
                    dp[c][k] = r;
                }
            }
            const size_t o = ((size_t)ze * N + wr(y0 + ey)) * N + wr(x0 + ex);
            // e1 = D3'v2 - D2'v3, e2 = D1'v3 - D3'v1, e3 = D2'v1 - D1'v2
            E(se, 0, ey, ex) = cscale(csub(dp[1][2], dp[2][1]), a.mu[o]);
            E(se, 1, ey, ex) = cscale(csub(dp[2][0], dp[0][2]), a.mu[N3 + o]);
            E(se, 2, ey, ex) = cscale(csub(dp[0][1], dp[1][0]), a.mu[2 * N3 + o]);
        }
    };
    // q(zq) = B v into Q slot sq, from v(zq) (V slot sv) and v(zq + 1) (V slot sf)
    auto make_q = [&](int sq, int sv, int sf) {
        for (int i = t; i < LE_X * LE_Y; i += LT_NT) {
            const int qx = i % LE_X, qy = i / LE_X;   // cell (x0 - 1 + qx, y0 - 1 + qy) = V local (qx, qy)
            C q = mk<C>(0, 0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const C u = V(sv, c, qy, qx);
                const C uf[3] = {V(sv, c, qy, qx + 1), V(sv, c, qy + 1, qx), V(sf, c, qy, qx)};
                C r = imul(cadd(uf[c], u), a.ha[c]);
#pragma unroll
                for (int j = 0; j < 3; ++j) r = cadd(r, cscale(csub(uf[j], u), a.B[c][j]));
                q = cadd(q, r);
            }
            Q(sq, qy, qx) = q;
        }
    };
    // w(z) on the tile: e(z) in E slot ec, e(z + 1) in en, q(z) in Q slot qc,
    // q(z - 1) in qp, v(z) in V slot vc
    auto make_w = [&](int ec, int en, int qc, int qp, int vc, int z) {
        if (t >= LT_X * LT_Y) return;
        const int tlx = t % LT_X, tly = t / LT_X;
        C df[3][3];   // df[c][k] = D^_k e_c
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const C e = E(ec, c, tly, tlx);
            const C ef[3] = {E(ec, c, tly, tlx + 1), E(ec, c, tly + 1, tlx), E(en, c, tly, tlx)};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                C r = imul(cadd(ef[k], e), a.ha[k]);
#pragma unroll
                for (int j = 0; j < 3; ++j) r = cadd(r, cscale(csub(ef[j], e), a.B[k][j]));
                df[c][k] = r;
            }
        }
        // w1 = D2 e3 - D3 e2, w2 = D3 e1 - D1 e3, w3 = D1 e2 - D2 e1
        C w[3] = {csub(df[2][1], df[1][2]), csub(df[0][2], df[2][0]), csub(df[1][0], df[0][1])};
        const C q = Q(qc, tly + 1, tlx + 1);
        const C qb[3] = {Q(qc, tly + 1, tlx), Q(qc, tly, tlx + 1), Q(qp, tly + 1, tlx + 1)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            C r = imul(cadd(qb[k], q), -a.ha[k]);
#pragma unroll
            for (int j = 0; j < 3; ++j) r = cadd(r, cscale(csub(qb[j], q), a.B[k][j]));
            const C v = V(vc, k, tly + 1, tlx + 1);
            w[k] = cadd(cadd(w[k], cscale(r, a.gamma)), cscale(v, a.shift));
        }
        const int x = x0 + tlx, y = y0 + tly;
        if (x < N && y < N) {
            const size_t o = ((size_t)z * N + y) * N + x;
#pragma unroll
            for (int k = 0; k < 3; ++k) Y[k * N3 + o] = mk<CS>(w[k].x, w[k].y);
        }
    };

    // prologue: v(z0 - 1), v(z0) -> e(z0), q(z0 - 1)
    fill(0, wr(z0 - 1));
    fill(1, z0);
    __syncthreads();
    make_e(0, 1, 0, z0);
    make_q(0, 0, 1);
    __syncthreads();
    int vc = 1, ec = 0, qp = 0;
    for (int z = z0; z < z1; ++z) {
        const int vn = vc ^ 1, en = ec ^ 1, qc = qp ^ 1;
        const int zn = (z + 1 == N) ? 0 : z + 1;
        fill(vn, zn);
        __syncthreads();
        make_e(en, vn, vc, zn);
        make_q(qc, vc, vn);
        __syncthreads();
        make_w(ec, en, qc, qp, vc, z);
        __syncthreads();
        vc = vn;
        ec = en;
        qp = qc;
    }
}

}  // namespace

template <class R, class S>
hipError_t launch_lattice(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                          const FieldList& fl) {
    if (!p.lattice || p.order != 2 || nb < 1 || p.N < 4) return hipErrorInvalidValue;
    LatArgs<R> a;
    a.X = X;
    a.Y = Y;
    a.mu = (const R*)mu;
    a.N = p.N;
    a.nb = nb;
    a.ntx = (p.N + LT_X - 1) / LT_X;
    a.nty = (p.N + LT_Y - 1) / LT_Y;
    for (int i = 0; i < 3; ++i) {
        a.ha[i] = (R)(0.5 * p.k[i]);
        for (int j = 0; j < 3; ++j) a.B[i][j] = (R)p.B[i][j];
    }
    a.gamma = (R)p.gamma;
    a.shift = (R)p.shift;
    a.fl = fl;
    // z chunks until the launch has about stencil_wgs workgroups; every
    // chunk holds at least 4 planes (each starts with two extra plane loads)
    const int tiles = a.ntx * a.nty * nb;
    int nzc = (p.stencil_wgs + tiles - 1) / tiles;
    nzc = std::max(1, std::min(nzc, p.N / 4));
    a.nzc = nzc;
    const size_t lds = (size_t)(2 * 3 + 2) * LE_Y * LE_X * sizeof(cplx<R>) +
                       (size_t)2 * 3 * LV_Y * LV_X * sizeof(cplx<S>);
    auto kern = lattice_fused_kernel<R, S>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * nzc)), dim3(LT_NT), lds, s, a);
    return hipGetLastError();
}

template hipError_t launch_lattice<float, float>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                                 const FieldList&);
template hipError_t launch_lattice<double, double>(const OpParams&, int, const void*, void*, const void*,
                                                   hipStream_t, const FieldList&);
template hipError_t launch_lattice<double, float>(const OpParams&, int, const void*, void*, const void*,
                                                  hipStream_t, const FieldList&);

}  // namespace mfd
