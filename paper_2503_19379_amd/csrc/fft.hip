// FFT solve of the preconditioner  T = (P + c I)^-1 R,  P = A A' + gamma B'B
// (Section 5.1 eq. (penalised_marix); Section 5.2, Alg 5.1).
//
// Every D_i is a Kronecker product of circulants, so the 3-D DFT diagonalises
// all of them at once (eq. (diag_of_circ) and the corollary after it).  With
// the forward transform u_hat(p) = sum_r u[r] exp(-2 pi i p r / N) the symbol of
// D_i at frequency p (theta = 2 pi p / N) is
//   d_i(p) = (e^{i theta} - 1) / h + i alpha_i (1 + e^{i theta}) / 2,
// and by Cor 4.4 (A A' + B'B = diag(L, L, L)) the 3 x 3 symbol of P is
//   P_hat(p) = s I + (gamma - 1) conj(d) d^T,   s = |d_1|^2 + |d_2|^2 + |d_3|^2.
// On a general lattice (Section 4.2) every D^_i = sum_j b_ji K_j + i L_i is
// still a polynomial in the grid shifts, so the same 3 x 3 form holds with
//   d_i(p) = sum_j B_ij kappa(p_j) + i alpha_i lambda(p_i),
// kappa and lambda the unit-step difference and average symbols along one
// axis and B_ij = N (A^-1)_ji.
// Alg 5.1 inverts a scalar diagonal; here the per-frequency block is rank-one
// plus a multiple of I, so its inverse is closed form (Sherman-Morrison):
//   t_hat = ( r_hat - (gamma - 1) conj(d) (d^T r_hat) / (gamma s + c) ) / (s + c).
//
// Three kernels, each one read and one write of the block:
//   1. forward DFT along x and y of every (band, component, z) plane, in LDS;
//   2. per (band, y, run of x): forward DFT along z of all three components,
//      the 3 x 3 solve, inverse DFT along z;
//   3. inverse DFT along y and x of every plane.
// The 1-D transforms are in-place Stockham radix-4/2/3/5 passes: each pass
// stages its butterfly inputs in registers, synchronises, and writes the
// outputs back to the same LDS buffer.
#include "common.h"
#include "internal.h"

namespace mfd {

constexpr int first_radix(int m) {
    return (m % 4 == 0) ? 4 : (m % 2 == 0) ? 2 : (m % 3 == 0) ? 3 : (m % 5 == 0) ? 5 : 0;
}
constexpr bool fft_ok(int n) {
    while (n > 1) {
        int r = first_radix(n);
        if (!r) return false;
        n /= r;
    }
    return true;
}

// R-point DFT in place; forward uses exp(-2 pi i / R), inverse its conjugate.
template <int R, bool INV, class T>
__device__ __forceinline__ void dft(T* v) {
    using S = decltype(v[0].x);
    if constexpr (R == 2) {
        T a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        T t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        T t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        // -i t3 (forward) / +i t3 (inverse)
        T jt3 = INV ? mk<T>(-t3.y, t3.x) : mk<T>(t3.y, -t3.x);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, jt3);
        v[3] = csub(t1, jt3);
    } else if constexpr (R == 3) {
        const S h3 = (S)0.86602540378443864676;   // sin(2 pi / 3)
        T a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        T m = mk<T>(a.x - (S)0.5 * s.x, a.y - (S)0.5 * s.y);
        // forward: U1 = m - i h3 d, U2 = m + i h3 d
        T jd = INV ? mk<T>(-h3 * d.y, h3 * d.x) : mk<T>(h3 * d.y, -h3 * d.x);
        v[0] = cadd(a, s);
        v[1] = cadd(m, jd);
        v[2] = csub(m, jd);
    } else if constexpr (R == 5) {
        const S c1 = (S)0.30901699437494742410, c2 = (S)-0.80901699437494742410;
        const S s1 = (S)0.95105651629515357212, s2 = (S)0.58778525229247312917;
        T a = v[0];
        T be = cadd(v[1], v[4]), bm = csub(v[1], v[4]);
        T cd = cadd(v[2], v[3]), cm = csub(v[2], v[3]);
        T r1 = mk<T>(a.x + c1 * be.x + c2 * cd.x, a.y + c1 * be.y + c2 * cd.y);
        T r2 = mk<T>(a.x + c2 * be.x + c1 * cd.x, a.y + c2 * be.y + c1 * cd.y);
        T i1 = mk<T>(s1 * bm.x + s2 * cm.x, s1 * bm.y + s2 * cm.y);
        T i2 = mk<T>(s2 * bm.x - s1 * cm.x, s2 * bm.y - s1 * cm.y);
        // forward: U1 = r1 - i i1, U4 = r1 + i i1, U2 = r2 - i i2, U3 = r2 + i i2
        T j1 = INV ? mk<T>(-i1.y, i1.x) : mk<T>(i1.y, -i1.x);
        T j2 = INV ? mk<T>(-i2.y, i2.x) : mk<T>(i2.y, -i2.x);
        v[0] = mk<T>(a.x + be.x + cd.x, a.y + be.y + cd.y);
        v[1] = cadd(r1, j1);
        v[4] = csub(r1, j1);
        v[2] = cadd(r2, j2);
        v[3] = csub(r2, j2);
    }
}

// One Stockham pass of radix R on NL lines of length N held in LDS.
// addr(l, j) gives the LDS index of element j of line l.  LFAST: consecutive
// threads take consecutive lines (strided lines) rather than consecutive
// butterflies of one line (contiguous lines), to keep LDS accesses unit-stride.
template <class T, int N, int NL, int NT, bool INV, bool LFAST, int R, int NS, class Addr>
__device__ __forceinline__ void fft_pass(T* buf, const T* tw, Addr addr, int tid) {
    constexpr int M = N / R;
    constexpr int NB = NL * M;
    constexpr int PER = (NB + NT - 1) / NT;
    T v[PER][R];
    int dst[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int idx = tid + b * NT;
        if ((NB % NT == 0) || idx < NB) {
            const int l = LFAST ? idx % NL : idx / M;
            const int j = LFAST ? idx / NL : idx % M;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[addr(l, j + r * M)];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    T w = tw[k * r * (N / (NS * R))];
                    if (INV) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            dft<R, INV>(v[b]);
            dst[b] = (j / NS) * NS * R + k;
            dst[b] = dst[b] | (l << 16);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int idx = tid + b * NT;
        if ((NB % NT == 0) || idx < NB) {
            const int l = dst[b] >> 16;
            const int d = dst[b] & 0xffff;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[addr(l, d + r * NS)] = v[b][r];
        }
    }
    __syncthreads();
}

template <class T, int N, int NL, int NT, bool INV, bool LFAST, int NS, class Addr>
__device__ __forceinline__ void fft_lines(T* buf, const T* tw, Addr addr, int tid) {
    if constexpr (NS < N) {
        constexpr int R = first_radix(N / NS);
        fft_pass<T, N, NL, NT, INV, LFAST, R, NS>(buf, tw, addr, tid);
        fft_lines<T, N, NL, NT, INV, LFAST, NS * R>(buf, tw, addr, tid);
    }
}

constexpr int FFT_NT = 256;

// Global <-> LDS staging of CNT elements by NT threads: element i sits at LDS
// index i and at global index at(i).  Each thread issues the loads of a chunk
// (up to 16 elements) before its first LDS write; a rolled copy loop would
// wait for every load in turn, one memory round trip per element.
template <int CNT, int NT, class T, class At>
__device__ __forceinline__ void stage_in(T* buf, const T* src, At at, int tid) {
    constexpr int PE = (CNT + NT - 1) / NT;
    constexpr int CH = PE < 16 ? PE : 16;
#pragma unroll
    for (int q0 = 0; q0 < PE; q0 += CH) {
        T v[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int i = tid + (q0 + q) * NT;
            if (q0 + q < PE && (CNT % NT == 0 || i < CNT)) v[q] = src[at(i)];
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int i = tid + (q0 + q) * NT;
            if (q0 + q < PE && (CNT % NT == 0 || i < CNT)) buf[i] = v[q];
        }
    }
}

// The reverse: LDS reads of a chunk first, then its global stores.
template <int CNT, int NT, class T, class At>
__device__ __forceinline__ void stage_out(const T* buf, T* dst, At at, int tid) {
    constexpr int PE = (CNT + NT - 1) / NT;
    constexpr int CH = PE < 16 ? PE : 16;
#pragma unroll
    for (int q0 = 0; q0 < PE; q0 += CH) {
        T v[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int i = tid + (q0 + q) * NT;
            if (q0 + q < PE && (CNT % NT == 0 || i < CNT)) v[q] = buf[i];
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int i = tid + (q0 + q) * NT;
            if (q0 + q < PE && (CNT % NT == 0 || i < CNT)) dst[at(i)] = v[q];
        }
    }
}

// Threads of the plane kernel: about 16 elements per thread per pass.
constexpr int plane_nt(int N) {
    int t = (N * N / 16 + 63) / 64 * 64;
    return t < 256 ? 256 : (t > 1024 ? 1024 : t);
}

// Kernels 1 and 3: 2-D DFT along x and y of one N x N plane per workgroup.
template <class R, int N, bool INV>
__global__ __launch_bounds__(plane_nt(N)) void fft_plane_kernel(const cplx<R>* in, cplx<R>* out,
                                                                const cplx<R>* tw_g, FieldList fl) {
    using T = cplx<R>;
    constexpr int NT = plane_nt(N);
    extern __shared__ unsigned char smem_raw[];
    T* buf = reinterpret_cast<T*>(smem_raw);
    T* tw = buf + N * N;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)fl(blockIdx.x / (3 * N)) * 3 * N + blockIdx.x % (3 * N);
    const T* src = in + plane * N * N;
    T* dst = out + plane * N * N;
    for (int i = tid; i < N; i += NT) tw[i] = tw_g[i];
    stage_in<N * N, NT>(buf, src, [](int i) { return i; }, tid);
    __syncthreads();
    if (!INV) {
        fft_lines<T, N, N, NT, INV, false, 1>(buf, tw, [](int l, int j) { return l * N + j; }, tid);
        fft_lines<T, N, N, NT, INV, true, 1>(buf, tw, [](int l, int j) { return j * N + l; }, tid);
    } else {
        fft_lines<T, N, N, NT, INV, true, 1>(buf, tw, [](int l, int j) { return j * N + l; }, tid);
        fft_lines<T, N, N, NT, INV, false, 1>(buf, tw, [](int l, int j) { return l * N + j; }, tid);
    }
    stage_out<N * N, NT>(buf, dst, [](int i) { return i; }, tid);
}

// Grids whose N x N plane does not fit in LDS (N = 150): kernels 1 and 3 are
// each split into a pass along x and a pass along y.
//   x pass: XL consecutive x lines of one (band, component, z) plane (they are
//     contiguous in memory) per workgroup;
//   y pass: N y values of XB consecutive x columns of one plane per workgroup,
//     rows of XB cells read and written coalesced.
template <int N> constexpr int line_block(int cap) {
    int b = 1;
    for (int d = 1; d <= cap; ++d)
        if (N % d == 0) b = d;
    return b;
}
template <int N> constexpr int xl_lines() { return line_block<N>(16); }
template <int N> constexpr int yl_cols() { return line_block<N>(32); }

template <class R, int N, bool INV>
__global__ __launch_bounds__(FFT_NT) void fft_xlines_kernel(const cplx<R>* in, cplx<R>* out, const cplx<R>* tw_g,
                                                           FieldList fl) {
    using T = cplx<R>;
    constexpr int XL = xl_lines<N>();
    extern __shared__ unsigned char smem_raw[];
    T* buf = reinterpret_cast<T*>(smem_raw);   // [XL][N]
    T* tw = buf + XL * N;
    const int tid = threadIdx.x;
    constexpr int NCH = N / XL;                // line blocks per plane
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const size_t plane = (size_t)fl(bid / (3 * N * NCH)) * 3 * N + (bid / NCH) % (3 * N);
    const size_t off = plane * N * N + (size_t)(bid % NCH) * XL * N;
    for (int i = tid; i < N; i += FFT_NT) tw[i] = tw_g[i];
    stage_in<XL * N, FFT_NT>(buf, in + off, [](int i) { return i; }, tid);
    __syncthreads();
    fft_lines<T, N, XL, FFT_NT, INV, false, 1>(buf, tw, [](int l, int j) { return l * N + j; }, tid);
    stage_out<XL * N, FFT_NT>(buf, out + off, [](int i) { return i; }, tid);
}

template <class R, int N, bool INV>
__global__ __launch_bounds__(FFT_NT) void fft_ylines_kernel(const cplx<R>* in, cplx<R>* out, const cplx<R>* tw_g,
                                                           FieldList fl) {
    using T = cplx<R>;
    constexpr int XB = yl_cols<N>();
    extern __shared__ unsigned char smem_raw[];
    T* buf = reinterpret_cast<T*>(smem_raw);   // [N (y)][XB]
    T* tw = buf + N * XB;
    const int tid = threadIdx.x;
    constexpr int NXB = N / XB;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const size_t plane = (size_t)fl(bid / (3 * N * NXB)) * 3 * N + (bid / NXB) % (3 * N);
    const size_t off = plane * N * N + (size_t)(bid % NXB) * XB;
    for (int i = tid; i < N; i += FFT_NT) tw[i] = tw_g[i];
    auto at = [](int i) { return (i / XB) * N + i % XB; };
    stage_in<N * XB, FFT_NT>(buf, in + off, at, tid);
    __syncthreads();
    fft_lines<T, N, XB, FFT_NT, INV, true, 1>(buf, tw, [](int l, int j) { return j * XB + l; }, tid);
    stage_out<N * XB, FFT_NT>(buf, out + off, at, tid);
}

template <class R, int N>
static hipError_t split_plane(const cplx<R>* in, cplx<R>* out, const cplx<R>* tw, int nb, bool inv, hipStream_t s,
                              const FieldList& fl) {
    using T = cplx<R>;
    constexpr int XL = xl_lines<N>(), XB = yl_cols<N>();
    const size_t lx = (size_t)(XL * N + N) * sizeof(T), ly = (size_t)(N * XB + N) * sizeof(T);
    auto kx = inv ? fft_xlines_kernel<R, N, true> : fft_xlines_kernel<R, N, false>;
    auto ky = inv ? fft_ylines_kernel<R, N, true> : fft_ylines_kernel<R, N, false>;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)kx, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lx)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void*)ky, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ly)) != hipSuccess)
        return e;
    const unsigned gx = (unsigned)(nb * 3 * N * (N / XL)), gy = (unsigned)(nb * 3 * N * (N / XB));
    // forward: x then y; inverse: y then x (as the plane kernel)
    if (!inv) {
        hipLaunchKernelGGL(kx, dim3(gx), dim3(FFT_NT), lx, s, in, out, tw, fl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(ky, dim3(gy), dim3(FFT_NT), ly, s, (const T*)out, out, tw, fl);
    } else {
        hipLaunchKernelGGL(ky, dim3(gy), dim3(FFT_NT), ly, s, in, out, tw, fl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(kx, dim3(gx), dim3(FFT_NT), lx, s, (const T*)out, out, tw, fl);
    }
    return hipGetLastError();
}

template <class R>
struct SolveArgs {
    const cplx<R>* in;
    cplx<R>* out;
    const cplx<R>* tw;
    R inv_h, half_k[3], gm1, gamma, shift, scale;
    int K;             // stencil half-width (order 2K)
    R c[4], d[4];      // Table FD_1D, c divided by h
    R alpha[3];
    int lattice;       // general lattice: d_i from B and the unit-step symbols
    R cu[4];           // Table FD_1D c, unit step
    R B[3][3];         // B[i][j]: weight of the difference along grid axis j in D_i
    FieldList fl;
};

// Symbol of D_i at frequency p (theta = 2 pi p / N) for the 2K-point stencil:
//   d(p) = sum_s c_s (e^{i s theta} - e^{i (1-s) theta}) + i alpha sum_s d_s (e^{i s theta} + e^{i (1-s) theta}),
// with e^{i m theta} = conj(tw[m p mod N]).
template <class R, int N>
__device__ __forceinline__ cplx<R> symbol_2k(const cplx<R>* tw, int p, const SolveArgs<R>& a, int axis) {
    using T = cplx<R>;
    T diff = mk<T>(0, 0), avg = mk<T>(0, 0);
    for (int s = 1; s <= a.K; ++s) {
        T e1 = tw[(p * s) % N];
        T e0 = tw[((p * (1 - s)) % N + N) % N];
        e1.y = -e1.y;
        e0.y = -e0.y;
        diff = cadd(diff, cscale(csub(e1, e0), a.c[s - 1]));
        avg = cadd(avg, cscale(cadd(e1, e0), a.d[s - 1]));
    }
    const R al = a.alpha[axis];
    return mk<T>(diff.x - al * avg.y, diff.y + al * avg.x);
}

// Unit-step symbols along one axis at frequency p:
//   kap = sum_s c_s (e^{i s theta} - e^{i (1-s) theta}),  lam = sum_s d_s (e^{i s theta} + e^{i (1-s) theta}).
template <class R, int N>
__device__ __forceinline__ void symbol_parts(const cplx<R>* tw, int p, const SolveArgs<R>& a, cplx<R>& kap,
                                             cplx<R>& lam) {
    using T = cplx<R>;
    kap = mk<T>(0, 0);
    lam = mk<T>(0, 0);
    for (int s = 1; s <= a.K; ++s) {
        T e1 = tw[(p * s) % N];
        T e0 = tw[((p * (1 - s)) % N + N) % N];
        e1.y = -e1.y;
        e0.y = -e0.y;
        kap = cadd(kap, cscale(csub(e1, e0), a.cu[s - 1]));
        lam = cadd(lam, cscale(cadd(e1, e0), a.d[s - 1]));
    }
}

// Kernel 2: DFT along z, 3 x 3 symbol solve, inverse DFT along z, for XC
// consecutive x positions of one y row of one band.
template <class R, int N, int XC>
__global__ __launch_bounds__(FFT_NT) void fft_zsolve_kernel(SolveArgs<R> a) {
    using T = cplx<R>;
    extern __shared__ unsigned char smem_raw[];
    T* buf = reinterpret_cast<T*>(smem_raw);   // [3][N (z)][XC]
    T* tw = buf + 3 * N * XC;
    const int tid = threadIdx.x;
    constexpr int NXC = N / XC;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int xc0 = (bid % NXC) * XC;
    const int y = (bid / NXC) % N;
    const int band = a.fl(bid / (NXC * N));
    const size_t NN = (size_t)N * N, N3 = NN * N;
    const T* src = a.in + (size_t)band * 3 * N3 + (size_t)y * N + xc0;
    T* dst = a.out + (size_t)band * 3 * N3 + (size_t)y * N + xc0;
    for (int i = tid; i < N; i += FFT_NT) tw[i] = a.tw[i];
    // element i of buf: x run position i % XC, z = (i / XC) % N, component i / (XC N)
    auto at = [](int i) {
        return (size_t)(i / (XC * N)) * ((size_t)N * N * N) + (size_t)((i / XC) % N) * (N * N) + i % XC;
    };
    stage_in<3 * N * XC, FFT_NT>(buf, src, at, tid);
    __syncthreads();
    auto addr = [](int l, int j) { return (l / XC) * N * XC + j * XC + (l % XC); };
    fft_lines<T, N, 3 * XC, FFT_NT, false, true, 1>(buf, tw, addr, tid);
    // symbol solve at every (pz, y, x)
    for (int i = tid; i < N * XC; i += FFT_NT) {
        const int xc = i % XC, pz = i / XC;
        const int px = xc0 + xc;
        // e^{i theta} = conj(tw[p])
        T ex = tw[px], ey = tw[y], ez = tw[pz];
        ex.y = -ex.y; ey.y = -ey.y; ez.y = -ez.y;
        T d1, d2, d3;
        if (a.lattice) {
            T kp[3], lm[3], dd[3];
            symbol_parts<R, N>(tw, px, a, kp[0], lm[0]);
            symbol_parts<R, N>(tw, y, a, kp[1], lm[1]);
            symbol_parts<R, N>(tw, pz, a, kp[2], lm[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dd[c] = mk<T>(-a.alpha[c] * lm[c].y, a.alpha[c] * lm[c].x);
#pragma unroll
                for (int j = 0; j < 3; ++j) dd[c] = cadd(dd[c], cscale(kp[j], a.B[c][j]));
            }
            d1 = dd[0];
            d2 = dd[1];
            d3 = dd[2];
        } else if (a.K == 1) {
            d1 = mk<T>((ex.x - (R)1) * a.inv_h - a.half_k[0] * ex.y, ex.y * a.inv_h + a.half_k[0] * ((R)1 + ex.x));
            d2 = mk<T>((ey.x - (R)1) * a.inv_h - a.half_k[1] * ey.y, ey.y * a.inv_h + a.half_k[1] * ((R)1 + ey.x));
            d3 = mk<T>((ez.x - (R)1) * a.inv_h - a.half_k[2] * ez.y, ez.y * a.inv_h + a.half_k[2] * ((R)1 + ez.x));
        } else {
            d1 = symbol_2k<R, N>(tw, px, a, 0);
            d2 = symbol_2k<R, N>(tw, y, a, 1);
            d3 = symbol_2k<R, N>(tw, pz, a, 2);
        }
        const R s = cabs2(d1) + cabs2(d2) + cabs2(d3);
        T r1 = buf[i], r2 = buf[N * XC + i], r3 = buf[2 * N * XC + i];
        T dr = cmul(d1, r1);
        dr = cfma(dr, d2, r2);
        dr = cfma(dr, d3, r3);
        const R coef = a.gm1 / (a.gamma * s + a.shift);
        const R inv = a.scale / (s + a.shift);
        dr = cscale(dr, coef);
        // t_i = (r_i - conj(d_i) dr) * inv
        r1 = cscale(csub(r1, cmulc(d1, dr)), inv);
        r2 = cscale(csub(r2, cmulc(d2, dr)), inv);
        r3 = cscale(csub(r3, cmulc(d3, dr)), inv);
        buf[i] = r1;
        buf[N * XC + i] = r2;
        buf[2 * N * XC + i] = r3;
    }
    __syncthreads();
    fft_lines<T, N, 3 * XC, FFT_NT, true, true, 1>(buf, tw, addr, tid);
    stage_out<3 * N * XC, FFT_NT>(buf, dst, at, tid);
}

static int pick_xc(int N) {
    for (int xc : {16, 8, 4, 10, 2, 1})
        if (N % xc == 0) return xc;
    return 1;
}

template <class R, int N, int XC>
static hipError_t zsolve_launch(const SolveArgs<R>& a, int nb, hipStream_t s) {
    const size_t lds = (3 * N * XC + N) * sizeof(cplx<R>);
    auto kern = fft_zsolve_kernel<R, N, XC>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nb * N * (N / XC)), dim3(FFT_NT), lds, s, a);
    return hipGetLastError();
}

template <class R, int N>
static hipError_t precond_n(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                            const FieldList& fl) {
    if (fl.on && nb > 32) return hipErrorInvalidValue;
    using T = cplx<R>;
    constexpr size_t lds_plane = (size_t)(N * N + N) * sizeof(T);
    constexpr bool SPLIT = lds_plane > 160 * 1024;
    auto kf = fft_plane_kernel<R, N, false>;
    auto ki = fft_plane_kernel<R, N, true>;
    const int nplanes = nb * 3 * N;
    hipError_t e;
    if constexpr (SPLIT) {
        if ((e = split_plane<R, N>((const T*)Rin, (T*)Tout, (const T*)tw, nb, false, s, fl)) != hipSuccess) return e;
    } else {
        e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_plane);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)ki, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_plane);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kf, dim3(nplanes), dim3(plane_nt(N)), lds_plane, s, (const T*)Rin, (T*)Tout,
                           (const T*)tw, fl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    SolveArgs<R> a;
    a.in = (const T*)Tout;
    a.out = (T*)Tout;
    a.tw = (const T*)tw;
    a.inv_h = (R)(1.0 / p.h);
    for (int i = 0; i < 3; ++i) a.half_k[i] = (R)(0.5 * p.k[i]);
    a.gm1 = (R)(p.gamma - 1.0);
    a.gamma = (R)p.gamma;
    a.shift = (R)p.shift;
    a.scale = (R)(1.0 / ((double)N * N * N));
    a.fl = fl;
    a.K = p.order / 2;
    {
        double c[4], d[4];
        stencil_coefs(p.order, c, d);
        for (int q = 0; q < 4; ++q) {
            a.c[q] = (R)(c[q] / p.h);
            a.cu[q] = (R)c[q];
            a.d[q] = (R)d[q];
        }
        for (int i = 0; i < 3; ++i) {
            a.alpha[i] = (R)p.k[i];
            for (int j = 0; j < 3; ++j) a.B[i][j] = (R)diff_weight(p, i, j);
        }
        a.lattice = p.lattice;
    }
    const int xc = (p.fft_xc > 0 && N % p.fft_xc == 0 && p.fft_xc <= 16) ? p.fft_xc : pick_xc(N);
    switch (xc) {
        case 16: if constexpr (N % 16 == 0) e = zsolve_launch<R, N, 16>(a, nb, s); break;
        case 10: if constexpr (N % 10 == 0 && N % 4) e = zsolve_launch<R, N, 10>(a, nb, s); break;
        case 8: if constexpr (N % 8 == 0) e = zsolve_launch<R, N, 8>(a, nb, s); break;
        case 4: if constexpr (N % 4 == 0) e = zsolve_launch<R, N, 4>(a, nb, s); break;
        case 2: if constexpr (N % 2 == 0) e = zsolve_launch<R, N, 2>(a, nb, s); break;
        default: e = zsolve_launch<R, N, 1>(a, nb, s); break;
    }
    if (e != hipSuccess) return e;
    if constexpr (SPLIT) return split_plane<R, N>((const T*)Tout, (T*)Tout, (const T*)tw, nb, true, s, fl);
    hipLaunchKernelGGL(ki, dim3(nplanes), dim3(plane_nt(N)), lds_plane, s, (const T*)Tout, (T*)Tout, (const T*)tw,
                       fl);
    return hipGetLastError();
}

#define MFD_FFT_SIZES(X) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(100) X(120) X(128) X(150)

bool fft_plane_fits(int N, int real_bytes) { return (size_t)(N * N + N) * 2 * real_bytes <= 160 * 1024; }

bool fft_supported(int N, int real_bytes) {
    switch (N) {
#define CASE(n) case n: return fft_ok(n);
        MFD_FFT_SIZES(CASE)
#undef CASE
        default: return false;
    }
}

template <class R>
hipError_t launch_precond(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                          const FieldList& fl) {
    // x run -1: the register-resident passes (FP32 on cubic order-2 grids of
    // 16, 32 or 64; elsewhere the built-in x run)
    if constexpr (sizeof(R) == 4)
        if (p.fft_xc == -1 && reg_precond_ok(p)) return launch_precond_reg(p, nb, Rin, Tout, tw, s, fl);
    switch (p.N) {
#define CASE(n) case n: return precond_n<R, n>(p, nb, Rin, Tout, tw, s, fl);
        MFD_FFT_SIZES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_precond<float>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                          const FieldList&);
template hipError_t launch_precond<double>(const OpParams&, int, const void*, void*, const void*, hipStream_t,
                                           const FieldList&);

}  // namespace mfd
