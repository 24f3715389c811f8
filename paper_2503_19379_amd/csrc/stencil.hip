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
// One kernel, stencil_wave_kernel (below), HBM-bound in intent: v read once,
// w written once, mu read from HBM about once per launch (the bands of a
// strip run side by side and share it in L2).  Each lane keeps the z history
// of its cells in registers and marches through a chunk of z planes; in-plane
// neighbours come from lanes of the same wave and from the lane's own rows.
// Intermediates e = mu A'v and q = Bv never touch HBM.  At step t the plane
// v(t+1) is loaded and the lane forms e(t+1) and q(t) and finally w(t) from
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
    int N, nzc, zc, nb;
    // waves per (band, z chunk), strips of TY rows, whole rows
    // per wave (nseg = 0) or row segments of seg cells (nseg of them)
    int wps, nstrip, rpw, nseg, seg, nwaves;
    FieldList fl;
    cplx<R> cp[3], cm[3];
    cplx<R> gcp[3], gcm[3];   // gamma cp, gamma cm
    R gamma, shift;
};

// Barrier-free form: x neighbours are lanes of the same wave and come
// through ds_bpermute, and y neighbours are registers: each lane owns a strip
// of TY rows (plus the halo rows y0 - 1 and y0 + TY, whose e and q it
// recomputes) and marches in z.  No LDS is allocated and no wave waits for
// another, so the memory, FP64 and permute work of different waves overlap
// on a CU.  State carried from plane t to t + 1, per lane: v(t) on rows
// -1..TY (storage precision), e(t) on rows 0..TY, q(t-1) on rows 0..TY-1.
// At most 168 VGPRs: 3 waves per SIMD.
//
// Lanes and x.  For N <= 64 a wave holds rpw = 64 / N whole periodic rows
// (strips) side by side: lane l is x = l % N of strip l / N, and its x
// neighbours wrap inside its group of N lanes.  Above 64 a row is cut into
// nseg segments of at most 62 cells, one per wave, with a halo lane on each
// side (x0 - 1 and x0 + len): the segment's edge cells need q of the left one
// and e of the right one, which those lanes form from their own v and that of
// the edge cell.  Halo and spare lanes compute like the others (their other
// neighbour is arbitrary, and what depends on it is used by no stored cell)
// and store nothing.

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

// Grid: a.nwaves waves in workgroups of 4; wave g is wave g % wps of band
// (g / wps) % nb and z chunk g / (wps nb), so consecutive waves share a band
// and z chunk; a.nzc chunks of N / nzc planes, rounded.
// NC: the grid size as a compile-time constant (0: a.N at run time), which
// turns the index arithmetic into shifts and constant multiplies.
template <class R, class S, int TY, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void stencil_wave_kernel(
    StencilArgs<R, S> a) {
    using T = cplx<R>;
    using TS = cplx<S>;
    const int N = NC ? NC : a.N;
    const int lane = threadIdx.x & 63;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    // the wave index through readfirstlane: the compiler then knows it (and the
    // band, z chunk and plane offsets derived from it) to be wave-uniform and
    // keeps them in scalar registers
    const int gwave = bid * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (gwave >= a.nwaves) return;   // whole waves; no barrier follows
    const int wv = gwave % a.wps;
    const int rest = gwave / a.wps;
    const int band = rest % a.nb;
    const int zch = rest / a.nb;
    // every lane stores when whole rows fill the wave and its strips evenly
    constexpr bool FULL = NC && NC <= 64 && 64 % NC == 0 && (NC / TY) % (64 / NC) == 0;
    int x, strip, lm, lp;
    bool st;                          // this lane's cells are stored
    if (NC ? NC <= 64 : a.nseg == 0) {
        const int gi = lane / N, xl = lane - gi * N;
        strip = wv * a.rpw + gi;
        st = FULL || (gi < a.rpw && strip < a.nstrip);
        if (!st) strip = 0;
        x = xl;
        lm = gi * N + (xl == 0 ? N - 1 : xl - 1);
        lp = gi * N + (xl == N - 1 ? 0 : xl + 1);
    } else {
        const int sg = wv % a.nseg;
        strip = wv / a.nseg;
        const int x0 = sg * a.seg;
        const int len = min(a.seg, N - x0);
        x = x0 - 1 + min(lane, len + 1);
        x = x < 0 ? x + N : (x >= N ? x - N : x);
        st = lane >= 1 && lane <= len;
        lm = lane > 0 ? lane - 1 : 0;
        lp = lane < 63 ? lane + 1 : 63;
    }
    const int am = (lm & 63) * 4;                 // ds_bpermute address of the lane at x - 1
    const int ap = (lp & 63) * 4;                 // at x + 1
    const int y0 = strip * TY;
    const int z0 = zch * N / a.nzc;
    const int z1 = (zch + 1) * N / a.nzc;
    const unsigned NN = (unsigned)N * N;
    const unsigned N3 = NN * N;
    const size_t fo = (size_t)a.fl(band) * 3 * N3;
    const char* Xb = (const char*)(a.X + fo);     // per-lane offsets below stay 32-bit
    char* Yb = (char*)(a.Y + fo);
    const char* Mb = (const char*)a.mu;
    unsigned yo[TY + 2];                          // rows y0 - 1 .. y0 + TY (cell index in a plane)
#pragma unroll
    for (int r = 0; r < TY + 2; ++r) {
        int y = y0 - 1 + r;
        y = NC ? (y + NC) % NC : (y < 0 ? y + N : (y >= N ? y - N : y));
        yo[r] = (unsigned)(y * N + x);
    }

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
        const unsigned zo = (unsigned)(NC ? (z + NC) % NC : (z < 0 ? z + N : (z >= N ? z - N : z))) * NN;
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
                if (FULL || st) {
                    const unsigned o = (unsigned)t * NN + yo[r + 1];
                    *(TS*)(Yb + (size_t)(o * (unsigned)sizeof(TS))) = mk<TS>(w0.x, w0.y);
                    *(TS*)(Yb + (size_t)((N3 + o) * (unsigned)sizeof(TS))) = mk<TS>(w1.x, w1.y);
                    *(TS*)(Yb + (size_t)((2 * N3 + o) * (unsigned)sizeof(TS))) = mk<TS>(w2.x, w2.y);
                }
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

template <class R, class S>
static hipError_t launch_wave(StencilArgs<R, S> a, int target, hipStream_t s) {
    const int N = a.N;
    constexpr int TY = 2;   // every grid the library accepts is even
    if (N % TY || N < 4) return hipErrorInvalidValue;
    a.nstrip = N / TY;
    if (N <= 64) {
        a.nseg = 0;
        a.seg = N;
        a.rpw = 64 / N;
        a.wps = (a.nstrip + a.rpw - 1) / a.rpw;
    } else {
        a.nseg = (N + 61) / 62;
        a.seg = (N + a.nseg - 1) / a.nseg;
        a.rpw = 1;
        a.wps = a.nstrip * a.nseg;
    }
    // z chunks (of at least 8 planes; each re-reads two halo planes) until
    // the grid has `target` waves
    const size_t per = (size_t)a.wps * a.nb;
    a.nzc = (int)std::min<size_t>(std::max<size_t>((target + per - 1) / per, 1), (size_t)std::max(N / 8, 1));
    a.zc = 0;
    a.nwaves = (int)(per * a.nzc);
    dim3 grid((a.nwaves + 3) / 4);
    switch (N) {
#define WAVE_N(n) case n: hipLaunchKernelGGL((stencil_wave_kernel<R, S, TY, n>), grid, dim3(256), 0, s, a); break;
        WAVE_N(24) WAVE_N(32) WAVE_N(48) WAVE_N(64) WAVE_N(96)
#undef WAVE_N
        default: hipLaunchKernelGGL((stencil_wave_kernel<R, S, TY, 0>), grid, dim3(256), 0, s, a); break;
    }
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
    for (int i = 0; i < 3; ++i) {
        a.cp[i] = mk<cplx<R>>(1.0 / p.h, 0.5 * p.k[i]);
        a.cm[i] = mk<cplx<R>>(-1.0 / p.h, 0.5 * p.k[i]);
        a.gcp[i] = mk<cplx<R>>(p.gamma / p.h, 0.5 * p.gamma * p.k[i]);
        a.gcm[i] = mk<cplx<R>>(-p.gamma / p.h, 0.5 * p.gamma * p.k[i]);
    }
    a.gamma = (R)p.gamma;
    a.shift = (R)p.shift;
    return launch_wave<R, S>(a, p.stencil_wgs, s);
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
