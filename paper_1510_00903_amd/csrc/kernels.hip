// gfx950 kernels of the effective block algorithm for baryon-baryon correlators.
// Paper: H. Nemura, arXiv:1510.00903, Sec. 3 (effective blocks and the FFT
// correlation of Eq. (LN.pLLp.FFT)).
//
// Per time slice the host driver launches, on one stream:
//   k_blocks     step 1a: every block intermediate at every site        (site-local)
//   k_fft (x3)   step 1b: forward 3-D FFT of every component            (one pass per axis)
//   k_fft3d_grouped  step 1b fused with the grouped copy, one pass (small cubic lattices)
//   k_fft_xy + k_fft_z_grouped  step 1b for 24- and 32-point planes: plane pass, then
//                the z pass writing into the momentum groups
//   k_transpose_grouped  component-major [g][comp][q] -> momentum groups (GroupLayout;
//                lattices without a fused form)
//   k_pairs      step 2a: open-index sums of every pair of intermediates, per momentum (MFMA)
//   k_pair_combine  step 2a: channels as weighted sums of the pair products
//   k_fft (x3)   step 2b: inverse 3-D FFT of the 16 spin components per channel
//   k_finalize   normalisation and transpose to the output layout [r][spin]
#include "kernels.hpp"

#include <algorithm>

namespace bbc {

// floor(log2(m)) for m > 0 (0 for m == 0): the rescale 2^-e brings max|S| into [1, 2).
__device__ __forceinline__ int pow2_exponent(float m) {
    if (!(m > 0.0f)) return 0;
    int e;
    (void)frexpf(m, &e);
    return e - 1;
}

// Float-float arithmetic (the FP32 form's compensated inverse transform):
// addition by Knuth's TwoSum of the high parts with the low parts added into
// the error term, multiplication by the FMA TwoProd of the high parts plus the
// cross terms, both renormalised (Fast2Sum) so that |lo| <= ulp(hi) / 2.
// Multiplication by an integer is used only with +1 and -1 (exact).
// The steps use explicitly rounded operations (__fadd_rn, __fsub_rn, __fmul_rn)
// so that no multiply-add is contracted into them.
__device__ __forceinline__ ff operator+(ff a, ff b) {
    const float s = __fadd_rn(a.hi, b.hi);
    const float v = __fsub_rn(s, a.hi);
    float e = __fadd_rn(__fsub_rn(a.hi, __fsub_rn(s, v)), __fsub_rn(b.hi, v));
    e = __fadd_rn(e, __fadd_rn(a.lo, b.lo));
    const float h = __fadd_rn(s, e);
    return ff(h, __fsub_rn(e, __fsub_rn(h, s)));
}
__device__ __forceinline__ ff operator-(ff a) { return ff(-a.hi, -a.lo); }
__device__ __forceinline__ ff operator-(ff a, ff b) { return a + (-b); }
__device__ __forceinline__ ff operator*(ff a, ff b) {
    const float p = __fmul_rn(a.hi, b.hi);
    float e = fmaf(a.hi, b.hi, -p);
    e = fmaf(a.hi, b.lo, e);
    e = fmaf(a.lo, b.hi, e);
    const float h = __fadd_rn(p, e);
    return ff(h, __fsub_rn(e, __fsub_rn(h, p)));
}
__device__ __forceinline__ ff operator*(int k, ff a) { return ff((float)k * a.hi, (float)k * a.lo); }

template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
    return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T2> __device__ __forceinline__ void cfma(T2 &acc, T2 a, T2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

// ----------------------------------------------------------------------------
// Step 1a: block intermediates.
//
// For a sink baryon term with tensor eps(c_a c_b c_c) Gamma_1(mu_a mu_b) Gamma_2(g, mu_c)
// (Sec. 2, Eq. (FieldOperator_B); the octet fields have Gamma_1 = C g5, Gamma_2 = 1)
// and propagators S_a, S_b, S_c, with Gamma_1(mu, p1[mu]) = i^k1[mu] and
// Gamma_2(g, p2[g]) = i^k2[g] (monomial in the Dirac representation), the diquark tensor
//   Q(c_c; e_a, e_b) = sum_{c_a c_b} eps(c_a c_b c_c) sum_mu i^k1[mu]
//                      S_a[3mu + c_a][e_a] S_b[3 p1[mu] + c_b][e_b]
// gives G(g; e_a, e_b, e_c) = i^k2[g] sum_{c_c} Q(c_c; e_a, e_b) S_c[3 p2[g] + c_c][e_c].
// Every intermediate component is a sum of G values times powers of i over the
// source indices closed at this site; the host planner lists those terms (packed
// e_a | e_b << 4 | e_c << 8 | (factor -1) << 12 | (factor i) << 13) per component.
// Components come in patterns (BlockPatterns): runs sharing the spin structure
// and the flavours of the three roles; adjacent patterns with the same diquark
// (flavours of roles a, b and Gamma_1) reuse its tensor.
// One workgroup handles TS consecutive sites and one of NSPLIT interleaved
// shares of the components (the diquark tensor is rebuilt per share, which is
// cheap next to the components); both sink spins are produced.  LDS rows are
// padded by one element so that the TS sites of a wave fall in distinct banks.
// Site blocks are placed XCD-aware (consecutive blocks on one XCD), so the
// partial output lines of neighbouring blocks meet in the same L2.
// Output layout: I[(g * nc + comp) * V + x].
// ----------------------------------------------------------------------------
// v * i^k for a wave-uniform k
template <typename T2> __device__ __forceinline__ T2 rot_i(T2 v, int k) {
    if (k & 1) v = T2{-v.y, v.x};
    if (k & 2) v = T2{-v.x, -v.y};
    return v;
}

template <typename T, int TS, int NSPLIT, bool IMAG>
__global__ __launch_bounds__(256) void k_blocks(const typename cplx_t<T>::type *__restrict__ Sl,
                                                const typename cplx_t<T>::type *__restrict__ Ss,
                                                typename cplx_t<T>::type *__restrict__ I, int V, int nc, int g0,
                                                const BlockComp *__restrict__ comps,
                                                const uint32_t *__restrict__ terms, const BlockPatterns pt,
                                                const uint32_t *__restrict__ kmax, const SliceArgs *__restrict__ ia) {
    using T2 = typename cplx_t<T>::type;
    if (ia) {
        Sl = (const T2 *)ia->sl;
        Ss = (const T2 *)ia->ss;
    }
    __shared__ T2 sS[2][TS][145];
    __shared__ T2 sQ[TS][433];
    const int tid = threadIdx.x;
    const int nsb = (V + TS - 1) / TS;
    const int sb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (sb >= nsb) return;
    const int x0 = sb * TS;
    const int share = blockIdx.y;
    // FP32 form: exact power-of-two rescale of each flavour's slice
    T kl = T(1), ks = T(1);
    if (kmax) {
        kl = T(ldexp(1.0, -pow2_exponent(__uint_as_float(kmax[0]))));
        ks = T(ldexp(1.0, -pow2_exponent(__uint_as_float(kmax[1]))));
    }
    for (int i = tid; i < TS * 144; i += 256) {
        int s = i / 144, e = i - s * 144, x = x0 + s;
        T2 zl = T2{0, 0}, zs = T2{0, 0};
        if (x < V) { zl = Sl[(size_t)x * 144 + e]; zs = Ss[(size_t)x * 144 + e]; }
        sS[0][s][e] = T2{zl.x * kl, zl.y * kl};
        sS[1][s][e] = T2{zs.x * ks, zs.y * ks};
    }
    const int site = tid % TS;
    const int slot = tid / TS;
    constexpr int NSLOT = 256 / TS;
    for (int ip = 0; ip < pt.n; ++ip) {
        const BlockPattern &P = pt.p[ip];
        if (P.new_diquark) {
            __syncthreads();
            // diquark tensor of roles a (flavour qa) and b (flavour qb)
            const int qa = P.qa, qb = P.qb;
            for (int i = tid; i < TS * 432; i += 256) {
                int s = i / 432, r = i - s * 432;
                int cc = r / 144, ea = (r / 12) % 12, eb = r % 12;
                int c1 = (cc + 1) % 3, c2 = (cc + 2) % 3;
                T2 acc = T2{0, 0};
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const int nu = P.p1[mu];
                    T2 a1 = sS[qa][s][(3 * mu + c1) * 12 + ea], b2 = sS[qb][s][(3 * nu + c2) * 12 + eb];
                    T2 a2 = sS[qa][s][(3 * mu + c2) * 12 + ea], b1 = sS[qb][s][(3 * nu + c1) * 12 + eb];
                    T2 d = cmul(a1, b2);
                    T2 e = cmul(a2, b1);
                    T2 t = rot_i(T2{d.x - e.x, d.y - e.y}, P.k1[mu]);
                    acc.x += t.x;
                    acc.y += t.y;
                }
                sQ[s][r] = acc;
            }
            __syncthreads();
        }
        // pattern constants, wave-uniform (scalar registers)
        const int pc = __builtin_amdgcn_readfirstlane((int)P.qc);
        const int r0 = __builtin_amdgcn_readfirstlane(3 * (int)P.p2[g0]);
        const int r1 = __builtin_amdgcn_readfirstlane(3 * (int)P.p2[g0 + 1]);
        const int k20 = __builtin_amdgcn_readfirstlane((int)P.k2[g0]);
        const int k21 = __builtin_amdgcn_readfirstlane((int)P.k2[g0 + 1]);
        const int pbeg = __builtin_amdgcn_readfirstlane(P.begin), pend = __builtin_amdgcn_readfirstlane(P.end);
        const T2 *qs = &sQ[site][0];
        const T2 *s0 = &sS[pc][site][r0 * 12], *s1 = &sS[pc][site][r1 * 12];
        // one term for both sink spins: i^bit13 sum_c Q[c][ab] S_c[row + c][ec]
        auto term = [&](uint32_t code, T2 &g0v, T2 &g1v) {
            const int ab = code & 255, ec = (code >> 8) & 15;
            g0v = T2{0, 0};
            g1v = T2{0, 0};
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const T2 q = qs[cc * 144 + ab];
                cfma(g0v, q, s0[cc * 12 + ec]);
                cfma(g1v, q, s1[cc * 12 + ec]);
            }
            if (IMAG && ((code >> 13) & 1)) {
                g0v = T2{-g0v.y, g0v.x};
                g1v = T2{-g1v.y, g1v.x};
            }
        };
        auto add = [](T2 &acc, const T2 g, uint32_t code) {
            const T sg = (code >> 12) & 1 ? T(-1) : T(1);
            acc.x += sg * g.x;
            acc.y += sg * g.y;
        };
        // a pair of terms (every component has an even number of them): the LDS
        // reads of both issue together; they are added in their listed order
        auto pair = [&](uint32_t c0, uint32_t c1, T2 &acc0, T2 &acc1) {
            T2 ga0, ga1, gb0, gb1;
            term(c0, ga0, ga1);
            term(c1, gb0, gb1);
            add(acc0, ga0, c0);
            add(acc1, ga1, c0);
            add(acc0, gb0, c1);
            add(acc1, gb1, c1);
        };
        // each thread takes runs of CB consecutive components; the records of its
        // next run are in flight while it works on the current one
        constexpr int CB = 4;
        constexpr int CSTEP = NSLOT * NSPLIT * CB;
        auto fetch = [&](int c0, BlockComp *r) {
#pragma unroll
            for (int j = 0; j < CB; ++j) r[j] = comps[min(c0 + j, pend - 1)];   // past the end: unused
        };
        const int x = x0 + site;
        auto run = [&](int c0, const BlockComp *r) {
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int comp = c0 + j;
                if (comp >= pend) break;
                T2 acc0 = T2{0, 0}, acc1 = T2{0, 0};
                pair(r[j].t0, r[j].t1, acc0, acc1);
                for (uint32_t t = 2; t < r[j].n; t += 2) {
                    const uint2 cd = *(const uint2 *)&terms[r[j].rest + t - 2];
                    pair(cd.x, cd.y, acc0, acc1);
                }
                acc0 = rot_i(acc0, k20);
                acc1 = rot_i(acc1, k21);
                if (x < V) {
                    I[((size_t)comp) * V + x] = acc0;
                    I[((size_t)nc + comp) * V + x] = acc1;
                }
            }
        };
        BlockComp ra[CB], rb[CB];
        const int cfirst = pbeg + (share * NSLOT + slot) * CB;
        fetch(cfirst, ra);
        for (int c0 = cfirst; c0 < pend; c0 += 2 * CSTEP) {
            fetch(c0 + CSTEP, rb);
            run(c0, ra);
            if (c0 + CSTEP >= pend) break;
            fetch(c0 + 2 * CSTEP, ra);
            run(c0 + CSTEP, rb);
        }
    }
}

template <typename T, int TS, int NSPLIT>
static void launch_blocks_v(const typename cplx_t<T>::type *Sl, const typename cplx_t<T>::type *Ss,
                            typename cplx_t<T>::type *I, int V, int nc, int g0, const BlockComp *comps,
                            const uint32_t *terms, const BlockPatterns &pt, const uint32_t *kmax, hipStream_t st,
                            const SliceArgs *ia) {
    const long nsb = (V + TS - 1) / TS;
    const dim3 grid((unsigned)(8 * ((nsb + 7) / 8)), NSPLIT);
    if (pt.any_imag)      // some term carries a factor i (spin structures with imaginary entries)
        hipLaunchKernelGGL((k_blocks<T, TS, NSPLIT, true>), grid, dim3(256), 0, st, Sl, Ss, I, V, nc, g0, comps,
                           terms, pt, kmax, ia);
    else
        hipLaunchKernelGGL((k_blocks<T, TS, NSPLIT, false>), grid, dim3(256), 0, st, Sl, Ss, I, V, nc, g0, comps,
                           terms, pt, kmax, ia);
}

// Variants (each component of each site is formed by one thread in the same
// order, so every variant gives the same bits): sites per workgroup x component
// shares 0 = 4 x 2, 1 = 4 x 4, 2 = 8 x 2.
template <typename T>
void launch_blocks(const typename cplx_t<T>::type *Sl, const typename cplx_t<T>::type *Ss,
                   typename cplx_t<T>::type *I, int V, int nc, int g0, const BlockComp *comps,
                   const uint32_t *terms, const BlockPatterns &pt, const uint32_t *kmax, int variant,
                   hipStream_t st, const SliceArgs *ia) {
    switch (variant) {
    case 1: launch_blocks_v<T, 4, 4>(Sl, Ss, I, V, nc, g0, comps, terms, pt, kmax, st, ia); break;
    case 2: launch_blocks_v<T, 8, 2>(Sl, Ss, I, V, nc, g0, comps, terms, pt, kmax, st, ia); break;
    default: launch_blocks_v<T, 4, 2>(Sl, Ss, I, V, nc, g0, comps, terms, pt, kmax, st, ia); break;
    }
}

// ----------------------------------------------------------------------------
// FP32 form, input staging: largest |Re|, |Im| of one flavour's slice, as the
// bit pattern of a non-negative float (integer max is order independent, so
// the result does not depend on scheduling).
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_absmax(const float2 *__restrict__ S, long n, uint32_t *__restrict__ out,
                                                const SliceArgs *__restrict__ ia, int strange) {
    if (ia) S = (const float2 *)(strange ? ia->ss : ia->sl);
    __shared__ float wm[4];
    float m = 0.0f;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float2 v = S[i];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    // one atomic per workgroup (the maximum of its 4 waves): many workgroups
    // updating one word serialise on it
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(out, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

void launch_absmax(const float2 *Sl, const float2 *Ss, long n, uint32_t *kmax, hipStream_t st,
                   const SliceArgs *ia) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, kmax, 2);
    const int nblk = (int)std::min<long>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax, dim3(nblk), dim3(256), 0, st, Sl, n, kmax, ia, 0);
    hipLaunchKernelGGL(k_absmax, dim3(nblk), dim3(256), 0, st, Ss, n, kmax + 1, ia, 1);
}

__global__ void k_slice_args(SliceArgs *dst, SliceArgs v) {
    if (threadIdx.x == 0) *dst = v;
}

void launch_slice_args(SliceArgs *dst, const SliceArgs &v, hipStream_t st) {
    hipLaunchKernelGGL(k_slice_args, dim3(1), dim3(64), 0, st, dst, v);
}

// ----------------------------------------------------------------------------
// FFT: batched 1-D transforms along one axis, one line per thread, held in
// registers; Stockham autosort with radix 4/2/3 stages (compile-time length).
// X(k) = sum_j x(j) exp(sign * 2 pi i j k / N).
// ----------------------------------------------------------------------------
template <typename T2, int R> struct Dft;
template <typename T2> struct Dft<T2, 2> {
    __device__ static void run(T2 *v, int) {
        T2 a = v[0], b = v[1];
        v[0] = T2{a.x + b.x, a.y + b.y};
        v[1] = T2{a.x - b.x, a.y - b.y};
    }
};
template <typename T2> struct Dft<T2, 3> {
    __device__ static void run(T2 *v, int sgn) {
        using T = decltype(v[0].x);
        const T h = T(0.86602540378443864676);    // sqrt(3)/2
        T2 t{v[1].x + v[2].x, v[1].y + v[2].y};
        T2 u{v[1].x - v[2].x, v[1].y - v[2].y};
        T2 m{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
        T2 iu{-sgn * h * u.y, sgn * h * u.x};      // sign * i * sqrt(3)/2 * u
        v[0] = T2{v[0].x + t.x, v[0].y + t.y};
        v[1] = T2{m.x + iu.x, m.y + iu.y};
        v[2] = T2{m.x - iu.x, m.y - iu.y};
    }
};
template <typename T2> struct Dft<T2, 4> {
    __device__ static void run(T2 *v, int sgn) {
        T2 a{v[0].x + v[2].x, v[0].y + v[2].y}, b{v[0].x - v[2].x, v[0].y - v[2].y};
        T2 c{v[1].x + v[3].x, v[1].y + v[3].y}, e{v[1].x - v[3].x, v[1].y - v[3].y};
        T2 d{-sgn * e.y, sgn * e.x};               // sign * i * (v1 - v3)
        v[0] = T2{a.x + c.x, a.y + c.y};
        v[2] = T2{a.x - c.x, a.y - c.y};
        v[1] = T2{b.x + d.x, b.y + d.y};
        v[3] = T2{b.x - d.x, b.y - d.y};
    }
};

template <int Rem> struct NextRadix {
    static constexpr int value = (Rem % 4 == 0) ? 4 : ((Rem % 2 == 0) ? 2 : 3);
};

template <typename T2, int N, int Ns, int R>
__device__ __forceinline__ void stockham_stage(const T2 *in, T2 *out, const T2 *tw, int sgn) {
#pragma unroll
    for (int j = 0; j < N / R; ++j) {
        T2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[j + r * (N / R)];
        const int k = j % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r)
            if (k != 0) v[r] = cmul(v[r], tw[(r * k * (N / (Ns * R))) % N]);
        Dft<T2, R>::run(v, sgn);
        const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[idx + r * Ns] = v[r];
    }
}

template <typename T2, int N, int Ns> struct Stages {
    __device__ static void run(T2 *a, T2 *b, const T2 *tw, int sgn) {
        if constexpr (N / Ns > 1) {
            constexpr int R = NextRadix<N / Ns>::value;
            stockham_stage<T2, N, Ns, R>(a, b, tw, sgn);
            Stages<T2, N, Ns * R>::run(b, a, tw, sgn);
#pragma unroll
            for (int i = 0; i < N; ++i) a[i] = b[i];
        }
    }
};

template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft(typename cplx_t<T>::type *__restrict__ data, long nlines, int Lx,
                                             int Ly, int Lz, int axis, int sgn) {
    using T2 = typename cplx_t<T>::type;
    __shared__ T2 tw[N];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s, c;
        sincospi(2.0 * i / N, &s, &c);
        tw[i] = T2{T(c), T(sgn * s)};
    }
    __syncthreads();
    const long V = (long)Lx * Ly * Lz;
    const long lpc = V / N;                    // lines per component
    for (long line = (long)blockIdx.x * blockDim.x + threadIdx.x; line < nlines;
         line += (long)gridDim.x * blockDim.x) {
        const long comp = line / lpc;
        const long l = line - comp * lpc;
        long base, stride;
        if (axis == 0) { base = l * Lx; stride = 1; }
        else if (axis == 1) { long x = l % Lx, z = l / Lx; base = z * Lx * Ly + x; stride = Lx; }
        else { base = l; stride = (long)Lx * Ly; }
        T2 *p = data + comp * V + base;
        T2 a[N], b[N];
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = p[j * stride];
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int j = 0; j < N; ++j) p[j * stride] = a[j];
    }
}

// x and y transforms of whole (component, z) planes in LDS (Lx = Ly = N): P
// planes per workgroup, read and written with coalesced loads, one N-point
// line per thread and axis, rows padded to N + 1 against bank conflicts.
// Replaces two of the three axis passes.
template <typename T, int N, int P>
__global__ __launch_bounds__(256) void k_fft_xy(typename cplx_t<T>::type *__restrict__ data, long nplanes,
                                                int sgn) {
    using T2 = typename cplx_t<T>::type;
    static_assert(P * N <= 256, "one line per thread");
    __shared__ T2 buf[P][N][N + 1];
    __shared__ T2 tw[N];
    const int t = threadIdx.x;
    for (int i = t; i < N; i += 256) {
        double s, c;
        sincospi(2.0 * i / N, &s, &c);
        tw[i] = T2{T(c), T(sgn * s)};
    }
    const long plane0 = (long)blockIdx.x * P;
    T2 *base = data + plane0 * N * N;
    const int nvalid = (int)((nplanes - plane0 < P ? nplanes - plane0 : P) * N * N);
    constexpr int NL = (P * N * N + 255) / 256;    // elements per thread
    if constexpr (sizeof(T) == 4) {
        T2 v[NL];                                  // FP32: every load in flight before the LDS stores
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = t + 256 * i;
            if (e < nvalid) v[i] = base[e];
        }
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = t + 256 * i;
            if (e < nvalid) {
                const int p = e / (N * N), rem = e - p * N * N;
                buf[p][rem / N][rem % N] = v[i];
            }
        }
    } else {                                       // FP64: the register budget goes to the lines
        for (int e = t; e < nvalid; e += 256) {
            const int p = e / (N * N), rem = e - p * N * N;
            buf[p][rem / N][rem % N] = base[e];
        }
    }
    __syncthreads();
    T2 a[N], b[N];
    const int p = t / N, l = t % N;
    const bool line = t < P * N;
    if (line) {                                    // x line: plane p, row y = l
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = buf[p][l][j];
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int j = 0; j < N; ++j) buf[p][l][j] = a[j];
    }
    __syncthreads();
    if (line) {                                    // y line: plane p, column x = l
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = buf[p][j][l];
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int j = 0; j < N; ++j) buf[p][j][l] = a[j];
    }
    __syncthreads();
    for (int e = t; e < nvalid; e += 256) {
        const int pp = e / (N * N), rem = e - pp * N * N;
        base[e] = buf[pp][rem / N][rem % N];
    }
}

// Planes per workgroup: variant 0 fills up to 80 KB of LDS (one line per
// thread at most), variant 1 takes half as many (smaller workgroups, more of
// them per CU).  The transforms are the same either way.
template <typename T, int N, int PV>
static void fft_xy_v(typename cplx_t<T>::type *data, long nplanes, int sgn, hipStream_t st) {
    using T2 = typename cplx_t<T>::type;
    constexpr int PL = 81920 / (N * (N + 1) * (int)sizeof(T2));     // planes within 80 KB of LDS
    constexpr int P0 = PL < 256 / N ? PL : 256 / N;
    constexpr int P = PV == 0 || P0 < 2 ? P0 : P0 / 2;
    hipLaunchKernelGGL((k_fft_xy<T, N, P>), dim3((unsigned)((nplanes + P - 1) / P)), dim3(256), 0, st, data, nplanes,
                       sgn);
}
template <typename T, int N>
static void fft_xy(typename cplx_t<T>::type *data, long nplanes, int sgn, int variant, hipStream_t st) {
    if (variant == 1) fft_xy_v<T, N, 1>(data, nplanes, sgn, st);
    else fft_xy_v<T, N, 0>(data, nplanes, sgn, st);
}

// Square planes with a plane pass: 24 and 32 points; 96 points in FP32 (one
// 96 x 97 plane, 74.5 KB of LDS, per workgroup).
template <typename T> constexpr bool plane_pass_fits(int n) {
    return n == 24 || n == 32 || (n == 96 && sizeof(T) == 4);
}
template <typename T>
static void plane_pass(typename cplx_t<T>::type *data, long nplanes, int n, int sgn, hipStream_t st,
                       int variant = 0) {
    if (n == 24) fft_xy<T, 24>(data, nplanes, sgn, variant, st);
    else if (n == 32) fft_xy<T, 32>(data, nplanes, sgn, variant, st);
    else if constexpr (sizeof(T) == 4) fft_xy<T, 96>(data, nplanes, sgn, 0, st);
}

// Long lines (N = N1 * N2) along one axis, without holding a whole line per
// thread: a tile of W lines adjacent in memory is staged in
// LDS ([point][line], coalesced loads and stores), then the two-factor form
//   X[k1 + N1 k2] = sum_j2 w_N2^(j2 k2) w_N^(j2 k1) sum_j1 x[j2 + N2 j1] w_N1^(j1 k1)
// runs as W*N2 inner N1-point transforms (with the twiddle w_N^(j2 k1)) and
// W*N1 outer N2-point transforms, each thread holding at most N1 values.
template <typename T, int N1, int N2, int W>
__global__ __launch_bounds__(256) void k_fft_lds(typename cplx_t<T>::type *__restrict__ data, long nlines, int Lx,
                                                 int Ly, int Lz, int axis, int sgn) {
    using T2 = typename cplx_t<T>::type;
    constexpr int N = N1 * N2;
    __shared__ T2 buf[N][W + 1];
    __shared__ T2 tw1[N1], tw2[N2], twN[N];
    const int t = threadIdx.x;
    for (int i = t; i < N; i += 256) {
        double s, c;
        sincospi(2.0 * i / N, &s, &c);
        twN[i] = T2{T(c), T(sgn * s)};
        if (i < N1) { sincospi(2.0 * i / N1, &s, &c); tw1[i] = T2{T(c), T(sgn * s)}; }
        if (i < N2) { sincospi(2.0 * i / N2, &s, &c); tw2[i] = T2{T(c), T(sgn * s)}; }
    }
    __shared__ long lbase[W];                      // first element of each line of the tile, -1 past the end
    const long V = (long)Lx * Ly * Lz;
    const long lpc = V / N;                        // lines per component
    const long l0 = (long)blockIdx.x * W;
    const long stride = axis == 0 ? 1 : axis == 1 ? Lx : (long)Lx * Ly;
    if (t < W) {
        const long l = l0 + t;
        long b = -1;
        if (l < nlines) {
            const long comp = l / lpc, m = l - comp * lpc;
            long base;
            if (axis == 0) base = m * Lx;
            else if (axis == 1) base = (m / Lx) * Lx * Ly + m % Lx;
            else base = m;
            b = comp * V + base;
        }
        lbase[t] = b;
    }
    __syncthreads();
    for (int e = t; e < N * W; e += 256) {
        int j, w;
        if (axis == 0) { w = e / N; j = e - w * N; } else { j = e / W; w = e - j * W; }
        const long b = lbase[w];
        if (b >= 0) buf[j][w] = data[b + j * stride];
    }
    __syncthreads();
    for (int u = t; u < W * N2; u += 256) {        // inner transforms over j1, then the twiddle
        const int w = u % W, j2 = u / W;
        T2 a[N1], b[N1];
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) a[j1] = buf[j2 + N2 * j1][w];
        Stages<T2, N1, 1>::run(a, b, tw1, sgn);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) buf[j2 + N2 * k1][w] = k1 == 0 ? a[0] : cmul(a[k1], twN[(j2 * k1) % N]);
    }
    __syncthreads();
    constexpr int NU = (W * N1 + 255) / 256;       // outer transforms per thread
    T2 r[NU][N2];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int u = t + 256 * i;
        if (u < W * N1) {
            const int w = u % W, k1 = u / W;
            T2 b[N2];
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) r[i][j2] = buf[j2 + N2 * k1][w];
            Stages<T2, N2, 1>::run(r[i], b, tw2, sgn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int u = t + 256 * i;
        if (u < W * N1) {
            const int w = u % W, k1 = u / W;
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) buf[k1 + N1 * k2][w] = r[i][k2];
        }
    }
    __syncthreads();
    for (int e = t; e < N * W; e += 256) {
        int j, w;
        if (axis == 0) { w = e / N; j = e - w * N; } else { j = e / W; w = e - j * W; }
        const long b = lbase[w];
        if (b >= 0) data[b + j * stride] = buf[j][w];
    }
}

template <typename T, int N1, int N2>
static void fft_axis_lds(typename cplx_t<T>::type *data, long ncomp, const int L[3], int axis, int sgn,
                         hipStream_t st) {
    using T2 = typename cplx_t<T>::type;
    constexpr int N = N1 * N2;
    // tile width: a power of two <= 64 with the tile within 72 KB of LDS
    constexpr int W = (N * 65 * (int)sizeof(T2) <= 73728) ? 64 : (N * 33 * (int)sizeof(T2) <= 73728) ? 32 : 16;
    const long V = (long)L[0] * L[1] * L[2];
    const long nlines = ncomp * (V / N);
    hipLaunchKernelGGL((k_fft_lds<T, N1, N2, W>), dim3((unsigned)((nlines + W - 1) / W)), dim3(256), 0, st, data,
                       nlines, L[0], L[1], L[2], axis, sgn);
}

bool fft_size_supported(int n) {
    switch (n) {
    case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
        return true;
    default:
        return false;
    }
}

template <typename T, int N>
static void fft_axis(typename cplx_t<T>::type *data, long ncomp, const int L[3], int axis, int sgn, hipStream_t st) {
    const long V = (long)L[0] * L[1] * L[2];
    const long nlines = ncomp * (V / N);
    hipLaunchKernelGGL((k_fft<T, N>), dim3(grid1d(nlines)), dim3(256), 0, st, data, nlines, L[0], L[1], L[2],
                       axis, sgn);
}

// 48-, 64- and 96-point lines: one line per thread in FP32 (fits the registers,
// most loads in flight); the two-factor LDS form (6 x 8, 8 x 8, 12 x 8) in FP64,
// where a whole line per thread would spill to scratch.
template <typename T, int N>
static void fft_axis_long(typename cplx_t<T>::type *data, long ncomp, const int L[3], int axis, int sgn,
                          hipStream_t st) {
    static_assert(N == 48 || N == 64 || N == 96, "long lines");
    if constexpr (sizeof(T) == 8) fft_axis_lds<T, N / 8, 8>(data, ncomp, L, axis, sgn, st);
    else fft_axis<T, N>(data, ncomp, L, axis, sgn, st);
}

template <typename T>
int launch_fft3d(typename cplx_t<T>::type *data, long ncomp, const int L[3], int sgn, hipStream_t st) {
    if (L[0] == L[1] && plane_pass_fits<T>(L[0])) {   // x and y in one plane pass, then z
        plane_pass<T>(data, ncomp * L[2], L[0], sgn, st);
        int n = 1;
        const int Lz = L[2];
        if (Lz > 1) {
            switch (Lz) {
            case 2: fft_axis<T, 2>(data, ncomp, L, 2, sgn, st); break;
            case 3: fft_axis<T, 3>(data, ncomp, L, 2, sgn, st); break;
            case 4: fft_axis<T, 4>(data, ncomp, L, 2, sgn, st); break;
            case 6: fft_axis<T, 6>(data, ncomp, L, 2, sgn, st); break;
            case 8: fft_axis<T, 8>(data, ncomp, L, 2, sgn, st); break;
            case 12: fft_axis<T, 12>(data, ncomp, L, 2, sgn, st); break;
            case 16: fft_axis<T, 16>(data, ncomp, L, 2, sgn, st); break;
            case 24: fft_axis<T, 24>(data, ncomp, L, 2, sgn, st); break;
            case 32: fft_axis<T, 32>(data, ncomp, L, 2, sgn, st); break;
            case 48: fft_axis_long<T, 48>(data, ncomp, L, 2, sgn, st); break;
            case 64: fft_axis_long<T, 64>(data, ncomp, L, 2, sgn, st); break;
            case 96: fft_axis_long<T, 96>(data, ncomp, L, 2, sgn, st); break;
            default: return -1;
            }
            ++n;
        }
        return n;
    }
    int n = 0;
    for (int axis = 0; axis < 3; ++axis) {
        if (L[axis] > 1) ++n;
        switch (L[axis]) {
        case 1: break;
        case 2: fft_axis<T, 2>(data, ncomp, L, axis, sgn, st); break;
        case 3: fft_axis<T, 3>(data, ncomp, L, axis, sgn, st); break;
        case 4: fft_axis<T, 4>(data, ncomp, L, axis, sgn, st); break;
        case 6: fft_axis<T, 6>(data, ncomp, L, axis, sgn, st); break;
        case 8: fft_axis<T, 8>(data, ncomp, L, axis, sgn, st); break;
        case 12: fft_axis<T, 12>(data, ncomp, L, axis, sgn, st); break;
        case 16: fft_axis<T, 16>(data, ncomp, L, axis, sgn, st); break;
        case 24: fft_axis<T, 24>(data, ncomp, L, axis, sgn, st); break;
        case 32: fft_axis<T, 32>(data, ncomp, L, axis, sgn, st); break;
        case 48: fft_axis_long<T, 48>(data, ncomp, L, axis, sgn, st); break;
        case 64: fft_axis_long<T, 64>(data, ncomp, L, axis, sgn, st); break;
        case 96: fft_axis_long<T, 96>(data, ncomp, L, axis, sgn, st); break;
        default: return -1;
        }
    }
    return n;
}

// ----------------------------------------------------------------------------
// Transpose [R][C] -> [C][R] through a padded LDS tile.
// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// Momentum groups.  The contraction pairs every momentum q with -q.  Momenta are
// packed into groups of G = 8 that are closed under q -> -q, and the
// momentum-space intermediates are stored group by group: per group and
// component c, the two sink spins g and the G momenta,
//   FP64: [group][c][g][G]      FP32: [group][c][G][g],
// so that every load of eight lanes fills whole 128-byte lines (FP64: one line
// per sink spin; FP32: one line holds both, and one 16-byte load fetches both
// sink spins of a momentum), and both sites of a pair (q and -q) read inside
// the same group.
// gpos[p] = (momentum held by position p, or -1 for a padding slot; lane of -q
// within the group).
// ----------------------------------------------------------------------------
// Element offset of (component c, sink spin g, lane j) within a group:
// c * 2G + j * S + g * SG.
template <typename T2> struct GroupLayout;
template <> struct GroupLayout<double2> {
    static constexpr int G = 8;
    static constexpr int S = 2;      // stride of the momentum lane
    static constexpr int SG = 1;     // stride of the sink spin
};
// FP32: spin-major inside a group line ([c][g][G]): the 8 momenta of one sink
// spin are 64 contiguous bytes, so a writer that holds one spin (the one-pass
// FFT) stores whole 64-byte sectors.
template <> struct GroupLayout<float2> {
    static constexpr int G = 8;
    static constexpr int S = 1;
    static constexpr int SG = 8;
};

// Tile: 64 positions x TC components x both sink spins through LDS; read along
// the (grouped) momenta, written as one contiguous run per group.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_grouped(const typename cplx_t<T>::type *__restrict__ in,
                                                           typename cplx_t<T>::type *__restrict__ out, int nc,
                                                           long V, long npos, const int2 *__restrict__ gpos) {
    using T2 = typename cplx_t<T>::type;
    using Ly = GroupLayout<T2>;
    constexpr int G = Ly::G;
    constexpr int TC = 16384 / (64 * sizeof(T2));   // 16 components (FP64) or 32 (FP32): 32 KB tile
    __shared__ T2 tile[2 * TC][65];
    const long p0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * TC;
    const int t = threadIdx.x;
    {
        const int pl = t & 63;
        const long p = p0 + pl;
        const int q = p < npos ? gpos[p].x : -1;
        for (int r = t >> 6; r < 2 * TC; r += 4) {
            const int g = r / TC, c = c0 + (r - g * TC);
            T2 v = T2{0, 0};
            if (q >= 0 && c < nc) v = in[((long)g * nc + c) * V + q];
            tile[r][pl] = v;
        }
    }
    __syncthreads();
    const int ncl = min(TC, nc - c0);               // components in this tile
    for (int e = t; e < 64 * 2 * TC; e += 256) {
        const int gi = e / (2 * TC * G), rem = e - gi * (2 * TC * G);
        const int cl = rem / (2 * G), w = rem - cl * (2 * G);
        const int j = (w % (G * Ly::S)) / Ly::S, g = (w / Ly::SG) % 2;
        const long p = p0 + gi * G + j;
        if (p < npos && cl < ncl)
            out[((p / G) * nc + c0) * 2 * G + rem] = tile[g * TC + cl][gi * G + j];
    }
}

template <typename T>
void launch_transpose_grouped(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, long V,
                              int ngroup, const int2 *gpos, hipStream_t st) {
    using T2 = typename cplx_t<T>::type;
    constexpr int G = GroupLayout<T2>::G;
    constexpr int TC = 16384 / (64 * sizeof(T2));
    const long npos = (long)ngroup * G;
    dim3 grid((unsigned)((npos + 63) / 64), (unsigned)((nc + TC - 1) / TC));
    hipLaunchKernelGGL((k_transpose_grouped<T>), grid, dim3(256), 0, st, in, out, nc, V, npos, gpos);
}

// ----------------------------------------------------------------------------
// Forward 3-D FFT of one component held whole in LDS (cubic lattices with
// N^3 complex numbers <= 64 KB), fused with the scatter into the momentum
// groups: one workgroup per (sink spin g, component c) reads the component's
// N^3 values once, transforms x, y and z in LDS (one N-point line per thread
// and axis, rows padded to N + 1 against bank conflicts), and writes every
// momentum to its group position.  Replaces three axis passes and the
// transpose for such lattices.
// ----------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft3d_grouped(const typename cplx_t<T>::type *__restrict__ in,
                                                       typename cplx_t<T>::type *__restrict__ out, int nc,
                                                       long npos, const int2 *__restrict__ gpos, int sgn) {
    using T2 = typename cplx_t<T>::type;
    using Ly = GroupLayout<T2>;
    constexpr int G = Ly::G;
    constexpr int V = N * N * N;
    constexpr int NP = N + 1;                      // padded row
    constexpr int NQ = (V + 8 + 255) / 256;        // output positions per thread (npos <= V + 8)
    static_assert(N * N <= 256, "one z line per thread");
    __shared__ T2 buf[N * N * NP];
    __shared__ T2 tw[N];
    const int t = threadIdx.x;
    // the two sink spins of a component run back to back on one XCD (consecutive
    // workgroup ids cycle over the 8 XCDs), so the halves of each output line they
    // write meet in that XCD's L2
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int g = j & 1, c = xcd * (int)(gridDim.x >> 4) + (j >> 1);
    if (c >= nc) return;
    const bool line = t < N * N;
    // issue every global load first: this thread's z line (x, y) = (t % N, t / N)
    // and the momenta of its output positions
    const T2 *src = in + ((long)g * nc + c) * V;
    T2 a[N], b[N];
    if (line) {
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = src[j * N * N + t];
    }
    int qv[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const long p = t + 256L * i;
        qv[i] = p < npos ? gpos[p].x : -2;
    }
    for (int i = t; i < N; i += 256) {
        double s, co;
        sincospi(2.0 * i / N, &s, &co);
        tw[i] = T2{T(co), T(sgn * s)};
    }
    __syncthreads();
    const int xt = t % N, yt = t / N;
    if (line) {
        Stages<T2, N, 1>::run(a, b, tw, sgn);          // z
#pragma unroll
        for (int j = 0; j < N; ++j) buf[(j * N + yt) * NP + xt] = a[j];
    }
    __syncthreads();
    if (line) {                                    // x line r = z * N + y, here r = t
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = buf[t * NP + j];
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int j = 0; j < N; ++j) buf[t * NP + j] = a[j];
    }
    __syncthreads();
    if (line) {                                    // y line (x, z) = (t % N, t / N)
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = buf[(yt * N + j) * NP + xt];
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int j = 0; j < N; ++j) buf[(yt * N + j) * NP + xt] = a[j];
    }
    __syncthreads();
    T2 *dst = out + (long)c * 2 * G + g * Ly::SG;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = qv[i];
        if (q == -2) break;                        // past the last position
        const long p = t + 256L * i;
        T2 v = T2{0, 0};
        if (q >= 0) v = buf[(q / N) * NP + q % N];
        dst[(p / G) * nc * 2 * G + (p % G) * Ly::S] = v;
    }
}

// ----------------------------------------------------------------------------
// Last (z) pass of the forward FFT fused with the copy into the momentum groups,
// for lattices whose x and y transforms ran as plane passes: each thread
// transforms one z line (kx, ky) of one (sink spin g, component c) in registers
// and writes its N momenta to their group positions (posof: momentum -> position).
// A group line holds q and -q (and in FP32 both sink spins), so a workgroup
// takes whole mirror pairs of rows: the rows ky are ordered 0, Ly/2, 1, Ly-1, 2,
// Ly-2, ... and a workgroup takes R consecutive ones (R even), which puts
// (kx, ky, kz) and (-kx, -ky, -kz) in the same workgroup.  A group line holds
// both sink spins of its momenta, so the two spins of a chunk are consecutive
// workgroups (they run together and complete the lines in L2).  All workgroups
// of a component run back to back on one XCD, so most group lines are
// completed by one pair of workgroups running together and leave L2 whole.
// Replaces the z axis pass and k_transpose_grouped.
// ----------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft_z_grouped(const typename cplx_t<T>::type *__restrict__ in,
                                                       typename cplx_t<T>::type *__restrict__ out, int nc, int Lx,
                                                       int Ly, int nchunk, int rows, const int *__restrict__ posof,
                                                       int sgn) {
    using T2 = typename cplx_t<T>::type;
    using Ly_ = GroupLayout<T2>;
    constexpr int G = Ly_::G;
    __shared__ T2 tw[N];
    const int t = threadIdx.x;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int per_c = 2 * nchunk;                   // (chunk, sink spin) per component
    const int c = xcd * (int)(gridDim.x / (8 * per_c)) + j / per_c;
    const int r = j - (j / per_c) * per_c;
    const int chunk = r >> 1, g = r & 1;
    for (int i = t; i < N; i += 256) {
        double sn, cs;
        sincospi(2.0 * i / N, &sn, &cs);
        tw[i] = T2{T(cs), T(sgn * sn)};
    }
    __syncthreads();
    if (c >= nc) return;
    const int slot = t / Lx, kx = t - slot * Lx;
    const int prow = chunk * rows + slot;
    if (slot >= rows || prow >= Ly) return;
    const int ky = prow == 0 ? 0 : prow == 1 ? Ly / 2 : ((prow & 1) ? Ly - (prow >> 1) : (prow >> 1));
    const int nxy = Lx * Ly, line = kx + Lx * ky;
    int pk[N];
#pragma unroll
    for (int k = 0; k < N; ++k) pk[k] = posof[line + k * nxy];
    const T2 *src = in + ((long)g * nc + c) * (long)nxy * N + line;
    T2 a[N], b[N];
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] = src[(long)k * nxy];
    Stages<T2, N, 1>::run(a, b, tw, sgn);
    T2 *dst = out + (long)c * 2 * G + g * Ly_::SG;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int p = pk[k];
        dst[(long)(p / G) * nc * 2 * G + (p % G) * Ly_::S] = a[k];
    }
}

// Last (z) pass for square 24- and 32-point planes, writing whole x-row runs.
// The momentum groups of these lattices come in runs (one per mirror pair of
// x-rows {(ky, kz), (-ky, -kz)}, whole groups; xrun[ky + Ly kz] = first group of
// the run), so the z lines of the y-row pair {w, Ly - w} (w = 0: {0, Ly/2}), all
// kx and both sink spins hold every momentum of their runs: one workgroup per
// (component, y-row pair) transforms those 4 Lx z lines (one per thread), keeps
// them in LDS, then writes each run as whole group lines (the 2G values of a
// (group, component) are contiguous), reading the LDS at the momentum each
// output position holds:
//   r != m: position 2 j -> (kx = j, row r), 2 j + 1 -> (kx = -j, row m);
//   r == m: 0 -> kx = 0, 1 -> kx = Lx/2, 2 j -> kx = j, 2 j + 1 -> kx = -j (j >= 1).
template <typename T, int LX, int N>
__global__ __launch_bounds__(4 * LX) void k_fft_z_runs(const typename cplx_t<T>::type *__restrict__ in,
                                                      typename cplx_t<T>::type *__restrict__ out, int nc,
                                                      const int *__restrict__ xrun, int sgn) {
    using T2 = typename cplx_t<T>::type;
    using Ly_ = GroupLayout<T2>;
    constexpr int G = Ly_::G, LY = LX, NXY = LX * LY, NT = 4 * LX;
    __shared__ T2 buf[2][2][N][LX];               // [sink spin][row][kz][kx]
    __shared__ T2 tw[N];
    const int t = threadIdx.x;
    constexpr int NW = LY / 2;                     // y-row pairs
    const int c = blockIdx.x / NW, w = blockIdx.x - c * NW;
    for (int i = t; i < N; i += NT) {
        double sn, cs;
        sincospi(2.0 * i / N, &sn, &cs);
        tw[i] = T2{T(cs), T(sgn * sn)};
    }
    const int ky0 = w, ky1 = w == 0 ? LY / 2 : LY - w;
    {
        const int kx = t % LX, row = (t / LX) & 1, g = t / (2 * LX);
        const T2 *src = in + ((long)g * nc + c) * (long)NXY * N + (row ? ky1 : ky0) * LX + kx;
        T2 a[N], b[N];
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = src[(long)k * NXY];
        __syncthreads();                           // twiddles
        Stages<T2, N, 1>::run(a, b, tw, sgn);
#pragma unroll
        for (int k = 0; k < N; ++k) buf[g][row][k][kx] = a[k];
    }
    __syncthreads();
    T2 *dst = out + (long)c * 2 * G;
    for (int ri = 0; ri < 2; ++ri) {
        const int ky = ri ? ky1 : ky0, kym = (LY - ky) % LY;
        const int rim = kym == ky0 ? 0 : 1;        // row index of the mirror y-row
        for (int kz = 0; kz < N; ++kz) {
            const int kzm = (N - kz) % N;
            const int r = ky + LY * kz, m = kym + LY * kzm;
            if (m < r) continue;                   // written from the mirror row
            const int g0 = xrun[r];
            const bool self = m == r;
            const int nval = (self ? LX : 2 * LX) * 2;
            for (int v = t; v < nval; v += NT) {
                const int s = v >> 1, gs = v & 1, j = s >> 1;
                int x, rw = ri, z = kz;
                if (self) {
                    x = s == 0 ? 0 : s == 1 ? LX / 2 : ((s & 1) ? LX - j : j);
                } else if (s & 1) {
                    x = (LX - j) % LX; rw = rim; z = kzm;
                } else {
                    x = j;
                }
                dst[(long)(g0 + s / G) * nc * 2 * G + (s % G) * Ly_::S + gs * Ly_::SG] = buf[gs][rw][z][x];
            }
        }
    }
}

template <typename T, int LX, int N>
static void fft_z_runs(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int *xrun,
                       hipStream_t st) {
    const long nwg = (long)nc * (LX / 2);
    hipLaunchKernelGGL((k_fft_z_runs<T, LX, N>), dim3((unsigned)nwg), dim3(4 * LX), 0, st, in, out, nc, xrun, -1);
}

template <typename T, int LX>
static bool fft_z_runs_lz(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, int Lz,
                          const int *xrun, hipStream_t st) {
    switch (Lz) {
    case 2: fft_z_runs<T, LX, 2>(in, out, nc, xrun, st); return true;
    case 3: fft_z_runs<T, LX, 3>(in, out, nc, xrun, st); return true;
    case 4: fft_z_runs<T, LX, 4>(in, out, nc, xrun, st); return true;
    case 6: fft_z_runs<T, LX, 6>(in, out, nc, xrun, st); return true;
    case 8: fft_z_runs<T, LX, 8>(in, out, nc, xrun, st); return true;
    case 12: fft_z_runs<T, LX, 12>(in, out, nc, xrun, st); return true;
    case 16: fft_z_runs<T, LX, 16>(in, out, nc, xrun, st); return true;
    case 24: fft_z_runs<T, LX, 24>(in, out, nc, xrun, st); return true;
    case 32: fft_z_runs<T, LX, 32>(in, out, nc, xrun, st); return true;
    default: return false;
    }
}

// ----------------------------------------------------------------------------
// One-pass forward 3-D FFT of cubic 32-point (or 24-point) lattices in FP32, written
// into the run-ordered momentum groups: one workgroup per (component, sink
// spin) reads the component once, with its L^2 z lines in registers (two per
// thread) and transformed there; the kz planes are then taken in two batches
// of L/2 planes, each closed under kz -> -kz (below), so that every x-row run
// lies in one batch: a batch's planes go to LDS, their x
// and y lines are transformed there, and the batch's runs are written as whole
// 64-byte spin sectors (GroupLayout<float2> is spin-major).  The z transform
// comes first here and last in the two-pass form, so the two differ by
// rounding only.  Replaces the plane pass and the z pass (two HBM round trips)
// for these lattices.
// ----------------------------------------------------------------------------
// Batches of L/2 planes each: A = {0, L/2} and kz = 1..h, L-h..L-1 (h = L/4 - 1),
// B = the rest (h+1..L/2-1 and L/2+1..L-h-1); both closed under kz -> -kz, and
// each batch's x (or y) lines are L^2 / 2 = one per thread.
template <int L>
__host__ __device__ constexpr int onepass_na() { return L / 4 - 1; }
// plane slot of kz in batch b (-1 if not in it), and the kz of slot p
template <int L>
__device__ __forceinline__ int onepass_slot(int b, int kz) {
    constexpr int h = onepass_na<L>();
    const bool inA = kz == 0 || kz == L / 2 || kz <= h || kz >= L - h;
    if (b == 0) {
        if (!inA) return -1;
        return kz == L / 2 ? 2 * h + 1 : (kz <= h ? kz : kz - L + 2 * h + 1);
    }
    if (inA) return -1;
    return kz < L / 2 ? kz - h - 1 : kz - h - 2;
}
template <int L>
__device__ __forceinline__ int onepass_kz(int b, int p) {
    constexpr int h = onepass_na<L>();
    if (b == 0) return p <= h ? p : (p <= 2 * h ? p + L - 2 * h - 1 : L / 2);
    return p < L / 2 - h - 1 ? p + h + 1 : p + h + 2;
}

template <int L>
__global__ __launch_bounds__(L * L / 2) void k_fft3d_onepass(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                             int nc, const int *__restrict__ xrun, int sgn) {
    using Ly = GroupLayout<float2>;
    constexpr int G = Ly::G;
    constexpr int NT = L * L / 2;                  // threads; thread t holds z lines t and t + NT
    constexpr int PA = L / 2, PB = L / 2;          // planes per batch
    constexpr int LP = L + 1;                      // padded row
    __shared__ float2 buf[PA][L][LP];
    __shared__ float2 tw[L];
    const int t = threadIdx.x;
    // the two sink spins of a component run back to back on one XCD
    const int xcd = blockIdx.x & 7, jb = blockIdx.x >> 3;
    const int g = jb & 1, c = xcd * (int)(gridDim.x >> 4) + (jb >> 1);
    if (c >= nc) return;                           // whole workgroup
    for (int i = t; i < L; i += NT) {
        double sn, cs;
        sincospi(2.0 * i / L, &sn, &cs);
        tw[i] = float2{(float)cs, (float)(sgn * sn)};
    }
    const float2 *src = in + ((long)g * nc + c) * (long)(L * L * L);
    float2 a0[L], a1[L], bt[L];
#pragma unroll
    for (int kz = 0; kz < L; ++kz) {
        a0[kz] = src[kz * L * L + t];
        a1[kz] = src[kz * L * L + t + NT];
    }
    __syncthreads();                               // twiddles
    Stages<float2, L, 1>::run(a0, bt, tw, sgn);
    Stages<float2, L, 1>::run(a1, bt, tw, sgn);
    const int x0 = t % L, y0 = t / L, x1 = (t + NT) % L, y1 = (t + NT) / L;
    float2 *dst = out + (long)c * 2 * G + g * Ly::SG;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int np = b == 0 ? PA : PB;
        if (b == 1) __syncthreads();               // batch A's runs written
#pragma unroll
        for (int kz = 0; kz < L; ++kz) {
            const int p = onepass_slot<L>(b, kz);
            if (p >= 0) {
                buf[p][y0][x0] = a0[kz];
                buf[p][y1][x1] = a1[kz];
            }
        }
        __syncthreads();
        for (int l = t; l < np * L; l += NT) {     // x lines (plane p, row y)
            const int p = l / L, y = l - p * L;
            float2 v[L], w[L];
#pragma unroll
            for (int x = 0; x < L; ++x) v[x] = buf[p][y][x];
            Stages<float2, L, 1>::run(v, w, tw, sgn);
#pragma unroll
            for (int x = 0; x < L; ++x) buf[p][y][x] = v[x];
        }
        __syncthreads();
        for (int l = t; l < np * L; l += NT) {     // y lines (plane p, column x)
            const int p = l / L, x = l - p * L;
            float2 v[L], w[L];
#pragma unroll
            for (int y = 0; y < L; ++y) v[y] = buf[p][y][x];
            Stages<float2, L, 1>::run(v, w, tw, sgn);
#pragma unroll
            for (int y = 0; y < L; ++y) buf[p][y][x] = v[y];
        }
        __syncthreads();
        // the runs of this batch's x-rows r = (ky, kz) with mirror m = (-ky, -kz) >= r:
        // position s of a run -> (kx, row) as in k_fft_z_runs
        for (int it = t; it < np * L * 2 * L; it += NT) {
            const int s = it % (2 * L), row = it / (2 * L);
            const int p = row / L, ky = row - p * L;
            const int kz = onepass_kz<L>(b, p);
            const int kym = (L - ky) % L, kzm = (L - kz) % L;
            const int r = ky + L * kz, m = kym + L * kzm;
            if (m < r) continue;                   // written from the mirror row
            const bool self = m == r;
            if (self && s >= L) continue;
            const int j = s >> 1;
            int x, yy = ky, pz = p;
            if (self) {
                x = s == 0 ? 0 : s == 1 ? L / 2 : ((s & 1) ? L - j : j);
            } else if (s & 1) {
                x = (L - j) % L; yy = kym; pz = onepass_slot<L>(b, kzm);
            } else {
                x = j;
            }
            dst[(long)(xrun[r] + s / G) * nc * 2 * G + (s % G) * Ly::S] = buf[pz][yy][x];
        }
    }
}

// Whether the one-pass form is used: FP32, cubic 32, run-ordered groups.  (At
// 24^3 it is correct but slower than the two passes: with 288 threads and one
// workgroup per CU its serial phases are not hidden; 2.26 ms per 52-channel slice.)
template <typename T> bool fft3d_onepass_fits(const int L[3]) {
    return sizeof(T) == 4 && L[0] == L[1] && L[1] == L[2] && L[0] == 32;
}

template <typename T>
int launch_fft3d_onepass(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                         const int *xrun, hipStream_t st) {
    if constexpr (sizeof(T) != 4) {
        return -1;
    } else {
        if (!fft3d_onepass_fits<T>(L) || !xrun) return -1;
        const dim3 grid((unsigned)(16 * ((nc + 7) / 8)));   // 8 XCDs x 2 spins x ceil(nc / 8)
        if (L[0] == 24)
            hipLaunchKernelGGL((k_fft3d_onepass<24>), grid, dim3(24 * 24 / 2), 0, st, in, out, nc, xrun, -1);
        else
            hipLaunchKernelGGL((k_fft3d_onepass<32>), grid, dim3(32 * 32 / 2), 0, st, in, out, nc, xrun, -1);
        return 0;
    }
}

// Whether the plane pass + fused z pass applies: Lx = Ly in {24, 32}, Lz with a
// register transform.
template <typename T> bool fft3d_zgrouped_fits(const int L[3]) {
    if (L[0] != L[1] || !plane_pass_fits<T>(L[0])) return false;
    switch (L[2]) {
    case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 24: case 32: return true;
    case 96: return sizeof(T) == 4;
    default: return false;
    }
}

template <typename T, int N>
static void fft_z_grouped(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, int Lx,
                          int Ly, const int *posof, hipStream_t st) {
    const int rows = (256 / Lx) / 2 * 2;           // whole mirror pairs of rows per workgroup
    const int nchunk = (Ly + rows - 1) / rows;
    const long per_xcd = (long)((nc + 7) / 8) * 2 * nchunk;   // both sink spins of each chunk
    hipLaunchKernelGGL((k_fft_z_grouped<T, N>), dim3((unsigned)(8 * per_xcd)), dim3(256), 0, st, in, out, nc, Lx,
                       Ly, nchunk, rows, posof, -1);
}

// Forward 3-D FFT of the intermediates into the momentum groups: x and y as
// plane passes in place on `in`, then the fused z pass.  Returns the number of
// kernels launched, or -1 if the lattice does not fit this form.
template <typename T>
int launch_fft3d_zgrouped(typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                          const int *posof, const int *xrun, int plane_variant, hipStream_t st) {
    if (!fft3d_zgrouped_fits<T>(L)) return -1;
    const long ncomp = 2L * nc;
    plane_pass<T>(in, ncomp * L[2], L[0], -1, st, plane_variant);
    if (xrun && L[2] <= 32) {                      // run-ordered groups: whole runs per workgroup
        if (L[0] == 24 && fft_z_runs_lz<T, 24>(in, out, nc, L[2], xrun, st)) return 2;
        if (L[0] == 32 && fft_z_runs_lz<T, 32>(in, out, nc, L[2], xrun, st)) return 2;
    }
    switch (L[2]) {
    case 2: fft_z_grouped<T, 2>(in, out, nc, L[0], L[1], posof, st); break;
    case 3: fft_z_grouped<T, 3>(in, out, nc, L[0], L[1], posof, st); break;
    case 4: fft_z_grouped<T, 4>(in, out, nc, L[0], L[1], posof, st); break;
    case 6: fft_z_grouped<T, 6>(in, out, nc, L[0], L[1], posof, st); break;
    case 8: fft_z_grouped<T, 8>(in, out, nc, L[0], L[1], posof, st); break;
    case 12: fft_z_grouped<T, 12>(in, out, nc, L[0], L[1], posof, st); break;
    case 16: fft_z_grouped<T, 16>(in, out, nc, L[0], L[1], posof, st); break;
    case 24: fft_z_grouped<T, 24>(in, out, nc, L[0], L[1], posof, st); break;
    case 32: fft_z_grouped<T, 32>(in, out, nc, L[0], L[1], posof, st); break;
    case 96:
        if constexpr (sizeof(T) == 4) { fft_z_grouped<T, 96>(in, out, nc, L[0], L[1], posof, st); break; }
        return -1;
    default: return -1;
    }
    return 2;
}

// Whether the fused single-pass form applies: cubic lattice, N^3 complex <= 64 KB.
template <typename T> bool fft3d_grouped_fits(const int L[3]) {
    using T2 = typename cplx_t<T>::type;
    if (L[0] != L[1] || L[1] != L[2]) return false;
    switch (L[0]) {
    case 4: case 6: case 8: case 12: case 16: break;
    default: return false;
    }
    return (long)L[0] * L[0] * L[0] * sizeof(T2) <= 65536;
}

template <typename T>
int launch_fft3d_grouped(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                         int ngroup, const int2 *gpos, hipStream_t st) {
    using T2 = typename cplx_t<T>::type;
    if (!fft3d_grouped_fits<T>(L)) return -1;
    const long npos = (long)ngroup * GroupLayout<T2>::G;
    const dim3 grid((unsigned)(16 * ((nc + 7) / 8)));     // 8 XCDs x 2 spins x ceil(nc / 8)
    switch (L[0]) {
    case 4: hipLaunchKernelGGL((k_fft3d_grouped<T, 4>), grid, dim3(256), 0, st, in, out, nc, npos, gpos, -1); break;
    case 6: hipLaunchKernelGGL((k_fft3d_grouped<T, 6>), grid, dim3(256), 0, st, in, out, nc, npos, gpos, -1); break;
    case 8: hipLaunchKernelGGL((k_fft3d_grouped<T, 8>), grid, dim3(256), 0, st, in, out, nc, npos, gpos, -1); break;
    case 12: hipLaunchKernelGGL((k_fft3d_grouped<T, 12>), grid, dim3(256), 0, st, in, out, nc, npos, gpos, -1); break;
    case 16: hipLaunchKernelGGL((k_fft3d_grouped<T, 16>), grid, dim3(256), 0, st, in, out, nc, npos, gpos, -1); break;
    default: return -1;
    }
    return 0;
}

// ----------------------------------------------------------------------------
// Step 2a: contraction in momentum space (Sec. 3, Eq. (LN.pLLp.FFT)), pair form.
//
// Every channel is a weighted sum of pair products (pairs.hpp)
//   P_p(q)_{a b a' b'} = sum_k X_p(q; a, ., k) Y_p(-q; b, ., k),
// a complex product of a (sink spin x outer spin) x k matrix at each site with
// the open source indices k = (k3, k4) contracted.  k_pairs computes every
// pair product once per momentum with the matrix cores; k_pair_combine forms
// the channels from them with fixed weights in a fixed order.
//
// MFMA operand layouts (measured on gfx950):
//   FP64 v_mfma_f64_4x4x4_4b (4 blocks, K = 4): A[b][i][k] in lane i + 4b + 16k,
//        B[b][k][j] in lane j + 4b + 16k, D[b][i][j] in lane j + 4b + 16i;
//   FP32 v_mfma_f32_4x4x1_16b (16 blocks, K = 1): A[b][i] and B[b][j] in lane
//        i + 4b (j + 4b), D[b][i][j] in lane j + 4b, register i.
// Blocks are momenta: FP64 a wave takes one group of 8 momenta as two sets of 4;
// FP32 a wave takes two groups (16 momenta).  Rows i and columns j are
// (sink spin g = i & 1, outer spin i >> 1), so with the grouped layout
// [c][momentum][g] every operand load of a wave reads whole 128-byte lines.
// A complex product takes two real products per part:
//   re += Ar Br + (-Ai) Bi,   im += Ar Bi + Ai Br.
// A task shares its row operand among up to 8 column views (partners), each
// with its own accumulators; shape 1 (8 x 2) runs as two 4 x 4 halves with two
// zero columns.  A wave runs one task; workgroup = (momentum unit, 4 tasks),
// all tasks of a unit back to back on one XCD so the unit's data stays in that
// XCD's L2.  Output P[group][pair][spin][G], spin = a + 2 (b + 2 (a' + 2 b')).
// ----------------------------------------------------------------------------
typedef double dmfma_acc;
typedef float fmfma4 __attribute__((ext_vector_type(4)));

// Component offset of a row (or column) value: the task's view, the lane's outer
// spin(s) and open index.
struct LaneView {
    int base;        // view base + outer-spin offsets of this lane's row/column
    int sk3, sk4;
};

__device__ __forceinline__ int outer_stride(const PView &v, bool a_prime) { return a_prime ? v.so3 : v.so4; }

// FP64: one task for NS sets of 4 momenta of a group of 8 (sets set0 ..
// set0 + NS - 1); PIPE: software-pipelined loads.
template <int NP, int SHAPE, int NS, bool PIPE>
__device__ __forceinline__ void pair_task64(const double2 *__restrict__ gb, double2 *__restrict__ pb,
                                            const PTask &T, int lane, const int mir[2], int set0) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int G = GroupLayout<double2>::G;
    constexpr int S = GroupLayout<double2>::S, SG = GroupLayout<double2>::SG;
    const int ij = lane & 3, blk = (lane >> 2) & 3, kl = lane >> 4;
    const int g = ij & 1, o = ij >> 1;
    // momentum slots of the row and column reads of this lane, per set
    int srow[NS], scol[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int m = blk + 4 * (set0 + st);
        srow[st] = T.row_site == 0 ? m : mir[st];
        scol[st] = T.row_site == 0 ? mir[st] : m;
    }
    // row: shape 0 -> outer spin o of the view's carried one; shape 1 -> a' = o, b' = half
    const int rbase = T.row.base + o * (SHAPE == 0 ? outer_stride(T.row, T.row_a) : T.row.so3);
    const int rso4 = T.row.so4;
    bool colvalid = true;
    int cbase[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (SHAPE == 0) cbase[p] = T.col[p].base + o * outer_stride(T.col[p], !T.row_a);
        else cbase[p] = T.col[p].base;
    }
    if (SHAPE == 1) colvalid = ij < 2;
    double acc[NP][NS][H][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int h = 0; h < H; ++h) acc[p][st][h][0] = acc[p][st][h][1] = 0.0;
    const int K = T.K;
    // Operands of one step of four k (lane kl takes k = k0 + kl): every lane loads
    // (lanes past K read the in-range k = 0 entry and then take zeros, so no branch
    // surrounds the loads).  Software-pipelined: the loads of step k0 + 4 are issued
    // before the products of step k0, so each wave keeps a step of loads in flight.
    auto load_step = [&](int k0, double2 (&av)[NS][H], double2 (&bv)[NP][NS]) {
        const int kk = k0 + kl;
        const bool valid = kk < K;
        const int k3 = valid ? (kk * T.inv) >> 16 : 0;
        const int k4 = valid ? kk - k3 * T.kd4 : 0;
        const int roff = rbase + k3 * T.row.sk3 + k4 * T.row.sk4;
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int h = 0; h < H; ++h) av[st][h] = gb[(unsigned)(roff + h * rso4) * (2 * G) + srow[st] * S + g * SG];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int coff = cbase[p] + k3 * T.col[p].sk3 + k4 * T.col[p].sk4;
#pragma unroll
            for (int st = 0; st < NS; ++st) bv[p][st] = gb[(unsigned)coff * (2 * G) + scol[st] * S + g * SG];
        }
        const bool zr = valid, zc = valid && colvalid;
#pragma unroll
        for (int st = 0; st < NS; ++st) {
#pragma unroll
            for (int h = 0; h < H; ++h) av[st][h] = zr ? av[st][h] : double2{0.0, 0.0};
#pragma unroll
            for (int p = 0; p < NP; ++p) bv[p][st] = zc ? bv[p][st] : double2{0.0, 0.0};
        }
    };
    auto mma_step = [&](const double2 (&av)[NS][H], const double2 (&bv)[NP][NS]) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const double2 a = av[st][h], b = bv[p][st];
                    double re = acc[p][st][h][0], im = acc[p][st][h][1];
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, re, 0, 0, 0);
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(-a.y, b.y, re, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.y, im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.x, im, 0, 0, 0);
                    acc[p][st][h][0] = re;
                    acc[p][st][h][1] = im;
                }
    };
    if constexpr (PIPE) {
        double2 av0[NS][H], bv0[NP][NS], av1[NS][H], bv1[NP][NS];
        load_step(0, av0, bv0);
        for (int k0 = 0; k0 < K; k0 += 8) {
            // a step past K reloads k = 0 (in range) and is never used
            load_step(k0 + 4 < K ? k0 + 4 : 0, av1, bv1);
            mma_step(av0, bv0);
            if (k0 + 4 >= K) break;
            load_step(k0 + 8 < K ? k0 + 8 : 0, av0, bv0);
            mma_step(av1, bv1);
        }
    } else {
        for (int k0 = 0; k0 < K; k0 += 4) {
            double2 av[NS][H], bv[NP][NS];
            load_step(k0, av, bv);
            mma_step(av, bv);
        }
    }
    // D lane (j = lane & 3, block, i = lane >> 4)
    const int j = lane & 3, i = lane >> 4;
    if (SHAPE == 1 && j >= 2) return;
    const int gR = i & 1, oR = i >> 1, gC = j & 1, oC = j >> 1;
    const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        int ap, bp;
        if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
        else { ap = oR; bp = h; }
        const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double2 *dst = pb + ((size_t)T.pair[p] * 16 + sp) * G;
#pragma unroll
            for (int st = 0; st < NS; ++st) dst[blk + 4 * (set0 + st)] = double2{acc[p][st][h][0], acc[p][st][h][1]};
        }
    }
}

// FP32: one task for two groups (16 momenta).  gb0/gb1 and pb0/pb1 are the
// groups' data and outputs; lanes of a missing second group load zeros and
// store nothing.
template <int NP, int SHAPE, bool PIPE>
__device__ __forceinline__ void pair_task32(const float2 *__restrict__ gb0, const float2 *__restrict__ gb1,
                                            float2 *__restrict__ pb0, float2 *__restrict__ pb1, bool has1,
                                            const PTask &T, int lane, int mir) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int G = GroupLayout<float2>::G;
    constexpr int S = GroupLayout<float2>::S, SG = GroupLayout<float2>::SG;
    const int ij = lane & 3, blk = lane >> 2;
    const int g = ij & 1, o = ij >> 1;
    const bool second = blk >= 8;
    const bool active = !second || has1;
    const float2 *gb = second ? gb1 : gb0;
    const int m = blk & 7;
    const int srow = T.row_site == 0 ? m : mir, scol = T.row_site == 0 ? mir : m;
    const int rbase = T.row.base + o * (SHAPE == 0 ? outer_stride(T.row, T.row_a) : T.row.so3);
    const int rso4 = T.row.so4;
    int cbase[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (SHAPE == 0) cbase[p] = T.col[p].base + o * outer_stride(T.col[p], !T.row_a);
        else cbase[p] = T.col[p].base;
    }
    const bool colvalid = active && (SHAPE == 0 || ij < 2);
    fmfma4 acc[NP][H][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int h = 0; h < H; ++h) acc[p][h][0] = acc[p][h][1] = fmfma4{0.f, 0.f, 0.f, 0.f};
    const int K = T.K;
    // Operands of one k: every lane loads (lanes of a missing second group read
    // the first), then inactive lanes take zeros.  Software-pipelined as in the
    // FP64 form: the loads of k + 1 are issued before the products of k.
    auto load_step = [&](int kk, float2 (&av)[H], float2 (&bv)[NP]) {
        const int k3 = (kk * T.inv) >> 16;
        const int k4 = kk - k3 * T.kd4;
        const int roff = rbase + k3 * T.row.sk3 + k4 * T.row.sk4;
#pragma unroll
        for (int h = 0; h < H; ++h) av[h] = gb[(unsigned)(roff + h * rso4) * (2 * G) + srow * S + g * SG];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int coff = cbase[p] + k3 * T.col[p].sk3 + k4 * T.col[p].sk4;
            bv[p] = gb[(unsigned)coff * (2 * G) + scol * S + g * SG];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) av[h] = active ? av[h] : float2{0.f, 0.f};
#pragma unroll
        for (int p = 0; p < NP; ++p) bv[p] = colvalid ? bv[p] : float2{0.f, 0.f};
    };
    auto mma_step = [&](const float2 (&av)[H], const float2 (&bv)[NP]) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const float2 a = av[h], b = bv[p];
                fmfma4 re = acc[p][h][0], im = acc[p][h][1];
                re = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.x, re, 0, 0, 0);
                re = __builtin_amdgcn_mfma_f32_4x4x1f32(-a.y, b.y, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.y, im, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.x, im, 0, 0, 0);
                acc[p][h][0] = re;
                acc[p][h][1] = im;
            }
    };
    if constexpr (PIPE) {
        float2 av0[H], bv0[NP], av1[H], bv1[NP];
        load_step(0, av0, bv0);
        for (int kk = 0; kk < K; kk += 2) {
            // a step past K reloads k = 0 (in range) and is never used
            load_step(kk + 1 < K ? kk + 1 : 0, av1, bv1);
            mma_step(av0, bv0);
            if (kk + 1 >= K) break;
            load_step(kk + 2 < K ? kk + 2 : 0, av0, bv0);
            mma_step(av1, bv1);
        }
    } else {
        for (int kk = 0; kk < K; ++kk) {
            float2 av[H], bv[NP];
            load_step(kk, av, bv);
            mma_step(av, bv);
        }
    }
    // D lane (j = lane & 3, block), register i
    const int j = lane & 3;
    if (!active || (SHAPE == 1 && j >= 2)) return;
    float2 *pb = second ? pb1 : pb0;
    const int gC = j & 1, oC = j >> 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gR = i & 1, oR = i >> 1;
        const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            int ap, bp;
            if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
            else { ap = oR; bp = h; }
            const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
            for (int p = 0; p < NP; ++p)
                pb[((size_t)T.pair[p] * 16 + sp) * G + m] = float2{acc[p][h][0][i], acc[p][h][1][i]};
        }
    }
}

// ----------------------------------------------------------------------------
// LDS-staged forms.  Direct operand loads give each 4-lane block (one momentum,
// rows (sink spin, outer spin)) two 16- or 8-byte pieces of two different
// components, so the L1 takes two accesses per quad of lanes and limits the
// kernel (counters: texture data unit about 98 % busy in FP32).  Here a wave
// first copies the whole group lines its operands need for one round of open
// indices into its own LDS area (global_load_lds_dwordx4: 16 contiguous bytes
// per lane, whole 64-byte quads), then reads the MFMA operands from LDS.  The
// products and their order are those of the direct forms, so the bits are too.
// PIPE: two LDS buffers, the copies of the next round in flight while the
// current one is multiplied.
// ----------------------------------------------------------------------------
constexpr int kStageMaxViews = 9;           // H + NP <= 9 operand views per open index

// s_waitcnt immediate that waits until at most n vector-memory operations are
// outstanding (expcnt and lgkmcnt left at their maxima).
__host__ __device__ constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

typedef __attribute__((address_space(3))) void lds_void;

// FP32: one task for two groups (16 momenta), KS (2 or 4) open indices per
// round.  Lines (128 B: one component, both sink spins of the group's 8 momenta):
// li = ((v KS + kr) 2 + group) 2 + outer spin for the V = H + NP views (row
// halves, then partners); wave load w fills lines 8w .. 8w + 7, i.e. two open
// indices of one view, so the view's offsets are wave-uniform; the two outer
// spins of a line pair sit 128 B apart (all 64 banks for one LDS read).  More
// open indices per round give each wave more products per copy round trip.
template <int NP, int SHAPE, bool PIPE, int KS>
__device__ __forceinline__ void pair_task32_lds(const float2 *__restrict__ gb0, const float2 *__restrict__ gb1,
                                                float2 *__restrict__ pb0, float2 *__restrict__ pb1, bool has1,
                                                const PTask &T, int lane, int mir, float4 *wlds) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int V = H + NP, NL = 4 * KS * V, WL = NL / 8;
    constexpr int G = GroupLayout<float2>::G;
    const int ij = lane & 3, blk = lane >> 2;
    const int g = ij & 1, o = ij >> 1;
    const bool second = blk >= 8;
    const bool active = !second || has1;
    const int m = blk & 7;
    const int srow = T.row_site == 0 ? m : mir, scol = T.row_site == 0 ? mir : m;
    const bool colvalid = active && (SHAPE == 0 || ij < 2);
    // this lane's line within a wave load: q = lane / 8 = (kr & 1, group, outer spin)
    const int q = lane >> 3, ld_o = q & 1, ld_g1 = (q >> 1) & 1, ld_kr = q >> 2;
    const float4 *gsrc = (const float4 *)(ld_g1 ? gb1 : gb0) + (lane & 7);
    const int K = T.K, nround = (K + KS - 1) / KS;
    auto issue = [&](int r, int buf) {
#pragma unroll
        for (int hk = 0; hk < KS / 2; ++hk) {
            const int kk0 = r * KS + 2 * hk + ld_kr;
            const int kk = kk0 < K ? kk0 : 0;              // past K: an in-range line, never read
            const int k3 = (kk * T.inv) >> 16, k4 = kk - k3 * T.kd4;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const PView &vw = v < H ? T.row : T.col[v - H];
                int ostr, base = vw.base;
                if (SHAPE == 0) ostr = v < H ? outer_stride(T.row, T.row_a) : outer_stride(vw, !T.row_a);
                else { ostr = v < H ? T.row.so3 : 0; if (v < H) base += v * T.row.so4; }
                const int comp = base + ld_o * ostr + k3 * vw.sk3 + k4 * vw.sk4;
                __builtin_amdgcn_global_load_lds((const void *)(gsrc + (size_t)(unsigned)comp * G),
                                                 (lds_void *)(wlds + (buf * NL + (v * (KS / 2) + hk) * 8) * 8), 16,
                                                 0, 0);
            }
        }
    };
    fmfma4 acc[NP][H][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int h = 0; h < H; ++h) acc[p][h][0] = acc[p][h][1] = fmfma4{0.f, 0.f, 0.f, 0.f};
    const int gl = second ? 1 : 0;
    auto compute = [&](int r, int buf) {
        const float2 *L2 = (const float2 *)(wlds + buf * NL * 8);
#pragma unroll
        for (int kr = 0; kr < KS; ++kr) {
            if (r * KS + kr >= K) break;
            float2 av[H], bv[NP];
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int li = ((h * KS + kr) * 2 + gl) * 2 + o;
                av[h] = L2[li * 16 + srow * GroupLayout<float2>::S + g * GroupLayout<float2>::SG];
                av[h] = active ? av[h] : float2{0.f, 0.f};
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int li = (((H + p) * KS + kr) * 2 + gl) * 2 + o;
                bv[p] = L2[li * 16 + scol * GroupLayout<float2>::S + g * GroupLayout<float2>::SG];
                bv[p] = colvalid ? bv[p] : float2{0.f, 0.f};
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const float2 a = av[h], b = bv[p];
                    fmfma4 re = acc[p][h][0], im = acc[p][h][1];
                    re = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.x, re, 0, 0, 0);
                    re = __builtin_amdgcn_mfma_f32_4x4x1f32(-a.y, b.y, re, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.y, im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.x, im, 0, 0, 0);
                    acc[p][h][0] = re;
                    acc[p][h][1] = im;
                }
        }
    };
    issue(0, 0);
    for (int r = 0; r < nround; ++r) {
        if constexpr (PIPE) {
            if (r + 1 < nround) {
                issue(r + 1, (r + 1) & 1);
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(WL));
            } else {
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            }
            compute(r, r & 1);
        } else {
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            compute(r, 0);
            if (r + 1 < nround) issue(r + 1, 0);
        }
    }
    // D lane (j = lane & 3, block), register i
    const int j = lane & 3;
    if (!active || (SHAPE == 1 && j >= 2)) return;
    float2 *pb = second ? pb1 : pb0;
    const int gC = j & 1, oC = j >> 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gR = i & 1, oR = i >> 1;
        const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            int ap, bp;
            if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
            else { ap = oR; bp = h; }
            const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
            for (int p = 0; p < NP; ++p)
                pb[((size_t)T.pair[p] * 16 + sp) * G + m] = float2{acc[p][h][0][i], acc[p][h][1][i]};
        }
    }
}

// FP64: one task for one group (both sets of 4 momenta), one round = 4 open
// indices (the MFMA's K).  Lines (256 B: one component, both sink spins of the
// group's 8 momenta): li = (v 4 + kl) 2 + outer spin; wave load w fills lines
// 4w .. 4w + 3, all of view v = w / 2, so the view's offsets are wave-uniform.
// Lines of outer spin 1 hold their two 128-byte halves swapped, so the 16 lanes
// of one LDS read phase (both outer spins, one set) hit all 64 banks.
template <int NP, int SHAPE, bool PIPE>
__device__ __forceinline__ void pair_task64_lds(const double2 *__restrict__ gb, double2 *__restrict__ pb,
                                                const PTask &T, int lane, const int mir[2], double2 *wlds) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int V = H + NP, NL = 8 * V;
    constexpr int G = GroupLayout<double2>::G;
    const int ij = lane & 3, blk = (lane >> 2) & 3, kl = lane >> 4;
    const int g = ij & 1, o = ij >> 1;
    int srow[2], scol[2];
#pragma unroll
    for (int st = 0; st < 2; ++st) {
        const int mm = blk + 4 * st;
        srow[st] = T.row_site == 0 ? mm : mir[st];
        scol[st] = T.row_site == 0 ? mir[st] : mm;
    }
    const bool colvalid = SHAPE == 0 || ij < 2;
    // this lane's line within a wave load: q = lane / 16 = (kl & 1, outer spin); the
    // wave load's parity gives kl >> 1
    const int ld_o = (lane >> 4) & 1, ld_kl = lane >> 5;
    const double2 *gsrc = gb + ((lane & 15) ^ (ld_o << 3));
    const int K = T.K, nround = (K + 3) / 4;
    auto issue = [&](int r, int buf) {
        int k3[2], k4[2];
#pragma unroll
        for (int hk = 0; hk < 2; ++hk) {
            const int kk0 = r * 4 + 2 * hk + ld_kl;
            const int kk = kk0 < K ? kk0 : 0;
            k3[hk] = (kk * T.inv) >> 16;
            k4[hk] = kk - k3[hk] * T.kd4;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const PView &vw = v < H ? T.row : T.col[v - H];
            int ostr, base = vw.base;
            if (SHAPE == 0) ostr = v < H ? outer_stride(T.row, T.row_a) : outer_stride(vw, !T.row_a);
            else { ostr = v < H ? T.row.so3 : 0; if (v < H) base += v * T.row.so4; }
#pragma unroll
            for (int hk = 0; hk < 2; ++hk) {
                const int comp = base + ld_o * ostr + k3[hk] * vw.sk3 + k4[hk] * vw.sk4;
                __builtin_amdgcn_global_load_lds((const void *)(gsrc + (size_t)(unsigned)comp * (2 * G)),
                                                 (lds_void *)(wlds + (buf * NL + (v * 2 + hk) * 4) * 16), 16, 0, 0);
            }
        }
    };
    double acc[NP][2][H][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int h = 0; h < H; ++h) acc[p][st][h][0] = acc[p][st][h][1] = 0.0;
    auto compute = [&](int r, int buf) {
        const double2 *L = wlds + buf * NL * 16;
        const bool valid = r * 4 + kl < K;
        double2 av[2][H], bv[NP][2];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int li = (h * 4 + kl) * 2 + o;
                av[st][h] = L[li * 16 + ((srow[st] * 2 + g) ^ (o << 3))];
                av[st][h] = valid ? av[st][h] : double2{0.0, 0.0};
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int li = ((H + p) * 4 + kl) * 2 + o;
                bv[p][st] = L[li * 16 + ((scol[st] * 2 + g) ^ (o << 3))];
                bv[p][st] = (valid && colvalid) ? bv[p][st] : double2{0.0, 0.0};
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int st = 0; st < 2; ++st)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const double2 a = av[st][h], b = bv[p][st];
                    double re = acc[p][st][h][0], im = acc[p][st][h][1];
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, re, 0, 0, 0);
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(-a.y, b.y, re, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.y, im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.x, im, 0, 0, 0);
                    acc[p][st][h][0] = re;
                    acc[p][st][h][1] = im;
                }
    };
    issue(0, 0);
    for (int r = 0; r < nround; ++r) {
        if constexpr (PIPE) {
            if (r + 1 < nround) {
                issue(r + 1, (r + 1) & 1);
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * V));
            } else {
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            }
            compute(r, r & 1);
        } else {
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            compute(r, 0);
            if (r + 1 < nround) issue(r + 1, 0);
        }
    }
    // D lane (j = lane & 3, block, i = lane >> 4)
    const int j = lane & 3, i = lane >> 4;
    if (SHAPE == 1 && j >= 2) return;
    const int gR = i & 1, oR = i >> 1, gC = j & 1, oC = j >> 1;
    const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        int ap, bp;
        if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
        else { ap = oR; bp = h; }
        const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double2 *dst = pb + ((size_t)T.pair[p] * 16 + sp) * G;
#pragma unroll
            for (int st = 0; st < 2; ++st) dst[blk + 4 * st] = double2{acc[p][st][h][0], acc[p][st][h][1]};
        }
    }
}

// FP64, one set of 4 momenta per wave (set0).  A set is closed under q -> -q
// (the mirror of group position p is p or p ^ 1), so the wave needs only the
// set's 128-byte half of each group line: li = (v 4 + kl) 2 + outer spin, wave
// load v fills the 8 lines of view v (lane / 8 = (kl, outer spin)); the two
// outer spins of a line pair sit 128 B apart, so a 16-lane LDS read phase hits
// all 64 banks.
template <int NP, int SHAPE, bool PIPE>
__device__ __forceinline__ void pair_task64_lds1(const double2 *__restrict__ gb, double2 *__restrict__ pb,
                                                 const PTask &T, int lane, int mir, int set0, double2 *wlds) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int V = H + NP, NL = 8 * V;
    constexpr int G = GroupLayout<double2>::G;
    const int ij = lane & 3, blk = (lane >> 2) & 3, kl = lane >> 4;
    const int g = ij & 1, o = ij >> 1;
    const int mm = blk + 4 * set0;
    const int srow = (T.row_site == 0 ? mm : mir) - 4 * set0, scol = (T.row_site == 0 ? mir : mm) - 4 * set0;
    const bool colvalid = SHAPE == 0 || ij < 2;
    const int q = lane >> 3, ld_o = q & 1, ld_kl = q >> 1;
    const double2 *gsrc = gb + 8 * set0 + (lane & 7);
    const int K = T.K, nround = (K + 3) / 4;
    auto issue = [&](int r, int buf) {
        const int kk0 = r * 4 + ld_kl;
        const int kk = kk0 < K ? kk0 : 0;                  // past K: an in-range line, never read
        const int k3 = (kk * T.inv) >> 16, k4 = kk - k3 * T.kd4;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const PView &vw = v < H ? T.row : T.col[v - H];
            int ostr, base = vw.base;
            if (SHAPE == 0) ostr = v < H ? outer_stride(T.row, T.row_a) : outer_stride(vw, !T.row_a);
            else { ostr = v < H ? T.row.so3 : 0; if (v < H) base += v * T.row.so4; }
            const int comp = base + ld_o * ostr + k3 * vw.sk3 + k4 * vw.sk4;
            __builtin_amdgcn_global_load_lds((const void *)(gsrc + (size_t)(unsigned)comp * (2 * G)),
                                             (lds_void *)(wlds + (buf * NL + v * 8) * 8), 16, 0, 0);
        }
    };
    double acc[NP][H][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int h = 0; h < H; ++h) acc[p][h][0] = acc[p][h][1] = 0.0;
    auto compute = [&](int r, int buf) {
        const double2 *L = wlds + buf * NL * 8;
        const bool valid = r * 4 + kl < K;
        double2 av[H], bv[NP];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int li = (h * 4 + kl) * 2 + o;
            av[h] = L[li * 8 + srow * 2 + g];
            av[h] = valid ? av[h] : double2{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int li = ((H + p) * 4 + kl) * 2 + o;
            bv[p] = L[li * 8 + scol * 2 + g];
            bv[p] = (valid && colvalid) ? bv[p] : double2{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const double2 a = av[h], b = bv[p];
                double re = acc[p][h][0], im = acc[p][h][1];
                re = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, re, 0, 0, 0);
                re = __builtin_amdgcn_mfma_f64_4x4x4f64(-a.y, b.y, re, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.y, im, 0, 0, 0);
                im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.x, im, 0, 0, 0);
                acc[p][h][0] = re;
                acc[p][h][1] = im;
            }
    };
    issue(0, 0);
    for (int r = 0; r < nround; ++r) {
        if constexpr (PIPE) {
            if (r + 1 < nround) {
                issue(r + 1, (r + 1) & 1);
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(V));
            } else {
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            }
            compute(r, r & 1);
        } else {
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            compute(r, 0);
            if (r + 1 < nround) issue(r + 1, 0);
        }
    }
    // D lane (j = lane & 3, block, i = lane >> 4)
    const int j = lane & 3, i = lane >> 4;
    if (SHAPE == 1 && j >= 2) return;
    const int gR = i & 1, oR = i >> 1, gC = j & 1, oC = j >> 1;
    const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        int ap, bp;
        if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
        else { ap = oR; bp = h; }
        const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            pb[((size_t)T.pair[p] * 16 + sp) * G + mm] = double2{acc[p][h][0], acc[p][h][1]};
    }
}

// FP64 staged per set: one wave per (task, set of 4 momenta), workgroups of 4
// waves, the workgroups of a group consecutive on one XCD.
template <bool PIPE>
__global__ __launch_bounds__(256) void k_pairs_lds64s(const double2 *__restrict__ Iq, double2 *__restrict__ P, int nc,
                                                      int ubase, int ucount, const int2 *__restrict__ gpos,
                                                      int ngroup, const PTask *__restrict__ tasks, int ntask,
                                                      int npair) {
    constexpr int G = GroupLayout<double2>::G;
    constexpr int BUF16 = 8 * kStageMaxViews * 8;          // 16-byte units per wave and buffer (9 KB)
    constexpr int NBUF = PIPE ? 2 : 1;
    __shared__ double2 lds[4 * NBUF * BUF16];
    const int nitem = ntask * 2;
    const int nchunk = (nitem + 3) >> 2;
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    const int P8 = (ucount + 7) >> 3;
    const int ul = xcd * P8 + jj / nchunk;
    const int chunk = jj - (jj / nchunk) * nchunk;
    if (ul >= ucount) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = chunk * 4 + wave;
    if (item >= nitem) return;
    const int t = item >> 1, set0 = item & 1;
    const int lane = threadIdx.x & 63;
    const int grp = ubase + ul;
    const double2 *g0 = Iq + (size_t)grp * nc * 2 * G;
    double2 *p0 = P + (size_t)grp * npair * 16 * G;
    double2 *wlds = lds + wave * NBUF * BUF16;
    const int mir = gpos[(size_t)grp * G + ((lane >> 2) & 3) + 4 * set0].y;
    const PTask &Tk = tasks[t];
    const int np = __builtin_amdgcn_readfirstlane(Tk.np);
    const int shape = __builtin_amdgcn_readfirstlane(Tk.shape);
#define BBC_PAIRS_CASE(SH, N) \
    case N: pair_task64_lds1<N, SH, PIPE>(g0, p0, Tk, lane, mir, set0, wlds); break;
    if (shape == 0) {
        switch (np) {
            BBC_PAIRS_CASE(0, 1) BBC_PAIRS_CASE(0, 2) BBC_PAIRS_CASE(0, 3) BBC_PAIRS_CASE(0, 4)
            BBC_PAIRS_CASE(0, 5) BBC_PAIRS_CASE(0, 6) BBC_PAIRS_CASE(0, 7) BBC_PAIRS_CASE(0, 8)
            default: break;
        }
    } else {
        switch (np) {
            BBC_PAIRS_CASE(1, 1) BBC_PAIRS_CASE(1, 2) BBC_PAIRS_CASE(1, 3) BBC_PAIRS_CASE(1, 4)
            default: break;
        }
    }
#undef BBC_PAIRS_CASE
}

// FP64 row tile per set of 4 momenta (PairTables::tiles): the H views of each of
// the tile's row views (up to 3) and the NP column views are staged
// through LDS per round of 4 open-index items, as in pair_task64_lds1; row r
// multiplies column p where its pair id is set (wave-uniform), so each product is
// formed with the operands, order and MFMA sequence of the one-row tasks (same
// bits), while a column view is loaded once for all rows of the tile.
constexpr int kTileMaxViews = 10;                  // R H + NP: FP64 3 rows x 6 (3) cols, FP32 3 x 4 (2)
template <int NP, int SHAPE>
__device__ __forceinline__ void pair_tile64(const double2 *__restrict__ gb, double2 *__restrict__ pb,
                                            const PTask &T, int lane, int mir, int set0, double2 *wlds) {
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int R = 3;                           // FP64 plans hold tiles of at most 3 rows
    constexpr int V = R * H + NP, NL = 8 * V;
    static_assert(V <= kTileMaxViews, "tile views");
    constexpr int G = GroupLayout<double2>::G;
    const int ij = lane & 3, blk = (lane >> 2) & 3, kl = lane >> 4;
    const int g = ij & 1, o = ij >> 1;
    const int mm = blk + 4 * set0;
    const int srow = (T.row_site == 0 ? mm : mir) - 4 * set0, scol = (T.row_site == 0 ? mir : mm) - 4 * set0;
    const bool colvalid = SHAPE == 0 || ij < 2;
    const int q = lane >> 3, ld_o = q & 1, ld_kl = q >> 1;
    const double2 *gsrc = gb + 8 * set0 + (lane & 7);
    const int K = T.K, nround = (K + 3) / 4;
    const int nrow = __builtin_amdgcn_readfirstlane(T.nrow);
    int pid[R][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        pid[0][p] = __builtin_amdgcn_readfirstlane(T.pair[p]);
#pragma unroll
        for (int rr = 1; rr < R; ++rr) pid[rr][p] = rr < nrow ? __builtin_amdgcn_readfirstlane(T.pairx[rr - 1][p]) : -1;
    }
    auto issue = [&](int r) {
        const int kk0 = r * 4 + ld_kl;
        const int kk = kk0 < K ? kk0 : 0;                  // past K: an in-range line, never read
        const int k3 = (kk * T.inv) >> 16, k4 = kk - k3 * T.kd4;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool isrow = v < R * H;
            if (isrow && v / H >= nrow) continue;           // no such row in this tile
            const PView &vw = v < H ? T.row : (isrow ? T.rowx[v / H - 1] : T.col[v - R * H]);
            int ostr, base = vw.base;
            if (SHAPE == 0) ostr = isrow ? outer_stride(vw, T.row_a) : outer_stride(vw, !T.row_a);
            else { ostr = isrow ? vw.so3 : 0; if (isrow) base += (v % H) * vw.so4; }
            const int comp = base + ld_o * ostr + k3 * vw.sk3 + k4 * vw.sk4;
            __builtin_amdgcn_global_load_lds((const void *)(gsrc + (size_t)(unsigned)comp * (2 * G)),
                                             (lds_void *)(wlds + v * 8 * 8), 16, 0, 0);
        }
    };
    double acc[R][NP][H][2];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < H; ++h) acc[rr][p][h][0] = acc[rr][p][h][1] = 0.0;
    auto compute = [&](int r) {
        const double2 *L = wlds;
        const bool valid = r * 4 + kl < K;
        double2 av[R][H], bv[NP];
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int li = ((rr * H + h) * 4 + kl) * 2 + o;
                av[rr][h] = L[li * 8 + srow * 2 + g];
                av[rr][h] = valid ? av[rr][h] : double2{0.0, 0.0};
            }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int li = ((R * H + p) * 4 + kl) * 2 + o;
            bv[p] = L[li * 8 + scol * 2 + g];
            bv[p] = (valid && colvalid) ? bv[p] : double2{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                if (pid[rr][p] < 0) continue;
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const double2 a = av[rr][h], b = bv[p];
                    double re = acc[rr][p][h][0], im = acc[rr][p][h][1];
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, re, 0, 0, 0);
                    re = __builtin_amdgcn_mfma_f64_4x4x4f64(-a.y, b.y, re, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.y, im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.x, im, 0, 0, 0);
                    acc[rr][p][h][0] = re;
                    acc[rr][p][h][1] = im;
                }
            }
    };
    for (int r = 0; r < nround; ++r) {
        issue(r);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        compute(r);
    }
    // D lane (j = lane & 3, block, i = lane >> 4)
    const int j = lane & 3, i = lane >> 4;
    if (SHAPE == 1 && j >= 2) return;
    const int gR = i & 1, oR = i >> 1, gC = j & 1, oC = j >> 1;
    const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        int ap, bp;
        if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
        else { ap = oR; bp = h; }
        const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
                if (pid[rr][p] >= 0)
                    pb[((size_t)pid[rr][p] * 16 + sp) * G + mm] = double2{acc[rr][p][h][0], acc[rr][p][h][1]};
    }
}

// FP32 row tile over two groups (16 momenta), 2 open indices per round:
// pair_task32_lds with up to 3 row views (same operands, order and MFMA
// sequence per product, so the same bits).
template <int NP, int SHAPE>
__device__ __forceinline__ void pair_tile32(const float2 *__restrict__ gb0, const float2 *__restrict__ gb1,
                                            float2 *__restrict__ pb0, float2 *__restrict__ pb1, bool has1,
                                            const PTask &T, int lane, int mir, float4 *wlds) {
    constexpr int KS = 2;
    constexpr int H = SHAPE == 1 ? 2 : 1;
    constexpr int R = 3;                           // FP32 plans hold tiles of at most 3 rows
    constexpr int V = R * H + NP, NL = 4 * KS * V;
    static_assert(V <= kTileMaxViews, "tile views");
    constexpr int G = GroupLayout<float2>::G;
    const int ij = lane & 3, blk = lane >> 2;
    const int g = ij & 1, o = ij >> 1;
    const bool second = blk >= 8;
    const bool active = !second || has1;
    const int m = blk & 7;
    const int srow = T.row_site == 0 ? m : mir, scol = T.row_site == 0 ? mir : m;
    const bool colvalid = active && (SHAPE == 0 || ij < 2);
    const int q = lane >> 3, ld_o = q & 1, ld_g1 = (q >> 1) & 1, ld_kr = q >> 2;
    const float4 *gsrc = (const float4 *)(ld_g1 ? gb1 : gb0) + (lane & 7);
    const int K = T.K, nround = (K + KS - 1) / KS;
    const int nrow = __builtin_amdgcn_readfirstlane(T.nrow);
    int pid[R][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        pid[0][p] = __builtin_amdgcn_readfirstlane(T.pair[p]);
#pragma unroll
        for (int rr = 1; rr < R; ++rr) pid[rr][p] = rr < nrow ? __builtin_amdgcn_readfirstlane(T.pairx[rr - 1][p]) : -1;
    }
    auto issue = [&](int r) {
        const int kk0 = r * KS + ld_kr;
        const int kk = kk0 < K ? kk0 : 0;                  // past K: an in-range line, never read
        const int k3 = (kk * T.inv) >> 16, k4 = kk - k3 * T.kd4;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool isrow = v < R * H;
            if (isrow && v / H >= nrow) continue;           // no such row in this tile
            const PView &vw = v < H ? T.row : (isrow ? T.rowx[v / H - 1] : T.col[v - R * H]);
            int ostr, base = vw.base;
            if (SHAPE == 0) ostr = isrow ? outer_stride(vw, T.row_a) : outer_stride(vw, !T.row_a);
            else { ostr = isrow ? vw.so3 : 0; if (isrow) base += (v % H) * vw.so4; }
            const int comp = base + ld_o * ostr + k3 * vw.sk3 + k4 * vw.sk4;
            __builtin_amdgcn_global_load_lds((const void *)(gsrc + (size_t)(unsigned)comp * G),
                                             (lds_void *)(wlds + v * 8 * 8), 16, 0, 0);
        }
    };
    fmfma4 acc[R][NP][H][2];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int h = 0; h < H; ++h) acc[rr][p][h][0] = acc[rr][p][h][1] = fmfma4{0.f, 0.f, 0.f, 0.f};
    const int gl = second ? 1 : 0;
    auto compute = [&](int r) {
        const float2 *L2 = (const float2 *)wlds;
#pragma unroll
        for (int kr = 0; kr < KS; ++kr) {
            if (r * KS + kr >= K) break;
            float2 av[R][H], bv[NP];
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int li = (((rr * H + h) * KS + kr) * 2 + gl) * 2 + o;
                    av[rr][h] = L2[li * 16 + srow * GroupLayout<float2>::S + g * GroupLayout<float2>::SG];
                    av[rr][h] = active ? av[rr][h] : float2{0.f, 0.f};
                }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int li = (((R * H + p) * KS + kr) * 2 + gl) * 2 + o;
                bv[p] = L2[li * 16 + scol * GroupLayout<float2>::S + g * GroupLayout<float2>::SG];
                bv[p] = colvalid ? bv[p] : float2{0.f, 0.f};
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    if (pid[rr][p] < 0) continue;
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        const float2 a = av[rr][h], b = bv[p];
                        fmfma4 re = acc[rr][p][h][0], im = acc[rr][p][h][1];
                        re = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.x, re, 0, 0, 0);
                        re = __builtin_amdgcn_mfma_f32_4x4x1f32(-a.y, b.y, re, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.y, im, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.x, im, 0, 0, 0);
                        acc[rr][p][h][0] = re;
                        acc[rr][p][h][1] = im;
                    }
                }
        }
    };
    for (int r = 0; r < nround; ++r) {
        issue(r);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        compute(r);
    }
    const int j = lane & 3;
    if (!active || (SHAPE == 1 && j >= 2)) return;
    float2 *pb = second ? pb1 : pb0;
    const int gC = j & 1, oC = j >> 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gR = i & 1, oR = i >> 1;
        const int a = T.row_site == 0 ? gR : gC, b = T.row_site == 0 ? gC : gR;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            int ap, bp;
            if (SHAPE == 0) { ap = T.row_a ? oR : oC; bp = T.row_a ? oC : oR; }
            else { ap = oR; bp = h; }
            const int sp = a + 2 * b + 4 * ap + 8 * bp;
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    if (pid[rr][p] >= 0)
                        pb[((size_t)pid[rr][p] * 16 + sp) * G + m] =
                            float2{acc[rr][p][h][0][i], acc[rr][p][h][1][i]};
        }
    }
}

// FP32 row tiles: one wave per (tile, unit of two groups), workgroups of 4
// waves, the workgroups of a unit consecutive on one XCD.
__global__ __launch_bounds__(256) void k_pairs_tiles32(const float2 *__restrict__ Iq, float2 *__restrict__ P, int nc,
                                                       int ubase, int ucount, const int2 *__restrict__ gpos,
                                                       int ngroup, const PTask *__restrict__ tiles, int ntile,
                                                       int npair) {
    constexpr int G = GroupLayout<float2>::G;
    constexpr int BUF16 = 4 * 2 * kTileMaxViews * 8;       // 16-byte units per wave (10 KB)
    __shared__ float4 lds[4 * BUF16];
    const int nchunk = (ntile + 3) >> 2;
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    const int P8 = (ucount + 7) >> 3;
    const int ul = xcd * P8 + jj / nchunk;
    const int chunk = jj - (jj / nchunk) * nchunk;
    if (ul >= ucount) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = chunk * 4 + wave;
    if (t >= ntile) return;
    const int lane = threadIdx.x & 63;
    const int grp0 = (ubase + ul) * 2;
    const bool has1 = grp0 + 1 < ngroup;
    const float2 *g0 = Iq + (size_t)grp0 * nc * 2 * G;
    const float2 *g1 = has1 ? g0 + (size_t)nc * 2 * G : g0;
    float2 *p0 = P + (size_t)grp0 * npair * 16 * G;
    float2 *p1 = has1 ? p0 + (size_t)npair * 16 * G : p0;
    float4 *wlds = lds + wave * BUF16;
    const int blk = lane >> 2;
    const int gg = (blk >= 8 && has1) ? grp0 + 1 : grp0;
    const int mir = gpos[(size_t)gg * G + (blk & 7)].y;
    const PTask &Tk = tiles[t];
    const int np = __builtin_amdgcn_readfirstlane(Tk.np);
    const int shape = __builtin_amdgcn_readfirstlane(Tk.shape);
#define BBC_TILE32_CASE(SH, N) \
    case N: pair_tile32<N, SH>(g0, g1, p0, p1, has1, Tk, lane, mir, wlds); break;
    if (shape == 0) {            // FP32 tiles: at most 4 columns (2 in shape 1)
        switch (np) {
            BBC_TILE32_CASE(0, 1) BBC_TILE32_CASE(0, 2) BBC_TILE32_CASE(0, 3) BBC_TILE32_CASE(0, 4)
            default: break;
        }
    } else {
        switch (np) {
            BBC_TILE32_CASE(1, 1) BBC_TILE32_CASE(1, 2)
            default: break;
        }
    }
#undef BBC_TILE32_CASE
}

// FP64 row tiles per set: one wave per (tile, set of 4 momenta), workgroups of
// 4 waves, the workgroups of a group consecutive on one XCD.
__global__ __launch_bounds__(256) void k_pairs_tiles64s(const double2 *__restrict__ Iq, double2 *__restrict__ P,
                                                        int nc, int ubase, int ucount,
                                                        const int2 *__restrict__ gpos, int ngroup,
                                                        const PTask *__restrict__ tiles, int ntile, int npair) {
    constexpr int G = GroupLayout<double2>::G;
    constexpr int BUF16 = 8 * kTileMaxViews * 8;           // 16-byte units per wave (10 KB)
    __shared__ double2 lds[4 * BUF16];
    const int nitem = ntile * 2;
    const int nchunk = (nitem + 3) >> 2;
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    const int P8 = (ucount + 7) >> 3;
    const int ul = xcd * P8 + jj / nchunk;
    const int chunk = jj - (jj / nchunk) * nchunk;
    if (ul >= ucount) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = chunk * 4 + wave;
    if (item >= nitem) return;
    const int t = item >> 1, set0 = item & 1;
    const int lane = threadIdx.x & 63;
    const int grp = ubase + ul;
    const double2 *g0 = Iq + (size_t)grp * nc * 2 * G;
    double2 *p0 = P + (size_t)grp * npair * 16 * G;
    double2 *wlds = lds + wave * BUF16;
    const int mir = gpos[(size_t)grp * G + ((lane >> 2) & 3) + 4 * set0].y;
    const PTask &Tk = tiles[t];
    const int np = __builtin_amdgcn_readfirstlane(Tk.np);
    const int shape = __builtin_amdgcn_readfirstlane(Tk.shape);
#define BBC_TILE_CASE(SH, N) \
    case N: pair_tile64<N, SH>(g0, p0, Tk, lane, mir, set0, wlds); break;
    if (shape == 0) {            // FP64 tiles: at most 4 columns (2 in shape 1)
        switch (np) {
            BBC_TILE_CASE(0, 1) BBC_TILE_CASE(0, 2) BBC_TILE_CASE(0, 3) BBC_TILE_CASE(0, 4)
            default: break;
        }
    } else {
        switch (np) {
            BBC_TILE_CASE(1, 1) BBC_TILE_CASE(1, 2)
            default: break;
        }
    }
#undef BBC_TILE_CASE
}

// One wave per task of a momentum unit (FP64: one group; FP32: two groups),
// operands staged through each wave's LDS area; workgroups of 4 waves, the
// workgroups of a unit consecutive on one XCD.
template <typename T, bool PIPE, int KS = 2>
__global__ __launch_bounds__(256) void k_pairs_lds(const typename cplx_t<T>::type *__restrict__ Iq,
                                                   typename cplx_t<T>::type *__restrict__ P, int nc, int ubase,
                                                   int ucount, const int2 *__restrict__ gpos, int ngroup,
                                                   const PTask *__restrict__ tasks, int ntask, int npair) {
    using T2 = typename cplx_t<T>::type;
    constexpr int G = GroupLayout<T2>::G;
    constexpr int GPU_ = sizeof(T) == 8 ? 1 : 2;
    // per wave and buffer: FP32 4 KS V lines of 128 B (KS open indices), FP64 8 V lines of 256 B (4)
    constexpr int BUF16 = sizeof(T) == 8 ? 8 * kStageMaxViews * 16 : 4 * KS * kStageMaxViews * 8;   // 16-byte units
    constexpr int NBUF = PIPE ? 2 : 1;
    __shared__ float4 lds[4 * NBUF * BUF16];
    const int nchunk = (ntask + 3) >> 2;
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    const int P8 = (ucount + 7) >> 3;
    const int ul = xcd * P8 + jj / nchunk;
    const int chunk = jj - (jj / nchunk) * nchunk;
    if (ul >= ucount) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = chunk * 4 + wave;
    if (t >= ntask) return;
    const int lane = threadIdx.x & 63;
    const int unit = ubase + ul;
    const int grp0 = unit * GPU_;
    const bool has1 = GPU_ == 2 && grp0 + 1 < ngroup;
    const T2 *g0 = Iq + (size_t)grp0 * nc * 2 * G;
    const T2 *g1 = has1 ? g0 + (size_t)nc * 2 * G : g0;
    T2 *p0 = P + (size_t)grp0 * npair * 16 * G;
    T2 *p1 = has1 ? p0 + (size_t)npair * 16 * G : p0;
    float4 *wlds = lds + wave * NBUF * BUF16;
    int mir[2];
    if constexpr (sizeof(T) == 8) {
        const int blk = (lane >> 2) & 3;
        mir[0] = gpos[(size_t)grp0 * G + blk].y;
        mir[1] = gpos[(size_t)grp0 * G + blk + 4].y;
    } else {
        const int blk = lane >> 2;
        const int gg = (blk >= 8 && has1) ? grp0 + 1 : grp0;
        mir[0] = gpos[(size_t)gg * G + (blk & 7)].y;
        mir[1] = 0;
    }
    const PTask &Tk = tasks[t];
    const int np = __builtin_amdgcn_readfirstlane(Tk.np);
    const int shape = __builtin_amdgcn_readfirstlane(Tk.shape);
#define BBC_PAIRL_CASE(SH, N)                                                                                  \
    case N:                                                                                                    \
        if constexpr (sizeof(T) == 8) pair_task64_lds<N, SH, PIPE>(g0, p0, Tk, lane, mir, (double2 *)wlds);   \
        else pair_task32_lds<N, SH, PIPE, KS>(g0, g1, p0, p1, has1, Tk, lane, mir[0], wlds);                 \
        break;
    if (shape == 0) {
        switch (np) {
            BBC_PAIRL_CASE(0, 1) BBC_PAIRL_CASE(0, 2) BBC_PAIRL_CASE(0, 3) BBC_PAIRL_CASE(0, 4)
            BBC_PAIRL_CASE(0, 5) BBC_PAIRL_CASE(0, 6) BBC_PAIRL_CASE(0, 7) BBC_PAIRL_CASE(0, 8)
            default: break;
        }
    } else {
        switch (np) {
            BBC_PAIRL_CASE(1, 1) BBC_PAIRL_CASE(1, 2) BBC_PAIRL_CASE(1, 3) BBC_PAIRL_CASE(1, 4)
            default: break;
        }
    }
#undef BBC_PAIRL_CASE
}

template <typename T, int SHAPE, int NP, int NS, bool PIPE>
__device__ __forceinline__ void pair_dispatch_np(const typename cplx_t<T>::type *g0, const typename cplx_t<T>::type *g1,
                                                 typename cplx_t<T>::type *p0, typename cplx_t<T>::type *p1,
                                                 bool has1, const PTask &Tk, int lane, const int mir[2], int set0) {
    if constexpr (sizeof(T) == 8) pair_task64<NP, SHAPE, NS, PIPE>(g0, p0, Tk, lane, mir, set0);
    else pair_task32<NP, SHAPE, PIPE>(g0, g1, p0, p1, has1, Tk, lane, mir[0]);
}

// One wave per (task, momentum part) of a momentum unit: FP64 units are one
// group, a wave takes NS of its two sets of 4 momenta (NS = 2: the whole group);
// FP32 units are two groups, a wave takes both.  Workgroups of 4 waves; the
// workgroups of a unit are consecutive on one XCD.
template <typename T, int NS, bool PIPE>
__global__ __launch_bounds__(256) void k_pairs(const typename cplx_t<T>::type *__restrict__ Iq,
                                               typename cplx_t<T>::type *__restrict__ P, int nc, int ubase,
                                               int ucount, const int2 *__restrict__ gpos, int ngroup,
                                               const PTask *__restrict__ tasks, int ntask, int npair) {
    using T2 = typename cplx_t<T>::type;
    constexpr int G = GroupLayout<T2>::G;
    constexpr int GPU_ = sizeof(T) == 8 ? 1 : 2;        // groups per unit
    constexpr int PARTS = sizeof(T) == 8 ? 2 / NS : 1;  // waves per task
    const int nitem = ntask * PARTS;
    const int nchunk = (nitem + 3) >> 2;
    const int xcd = blockIdx.x & 7, jj = blockIdx.x >> 3;
    const int P8 = (ucount + 7) >> 3;
    const int ul = xcd * P8 + jj / nchunk;
    const int chunk = jj - (jj / nchunk) * nchunk;
    if (ul >= ucount) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = chunk * 4 + wave;
    if (item >= nitem) return;
    const int t = PARTS == 1 ? item : item / PARTS;
    const int set0 = PARTS == 1 ? 0 : item - t * PARTS;
    const int lane = threadIdx.x & 63;
    const int unit = ubase + ul;
    const int grp0 = unit * GPU_;
    const bool has1 = GPU_ == 2 && grp0 + 1 < ngroup;
    const T2 *g0 = Iq + (size_t)grp0 * nc * 2 * G;
    const T2 *g1 = has1 ? g0 + (size_t)nc * 2 * G : g0;
    T2 *p0 = P + (size_t)grp0 * npair * 16 * G;
    T2 *p1 = has1 ? p0 + (size_t)npair * 16 * G : p0;
    int mir[2];
    if constexpr (sizeof(T) == 8) {
        const int blk = (lane >> 2) & 3;
        mir[0] = gpos[(size_t)grp0 * G + blk + 4 * set0].y;
        mir[1] = NS == 2 ? gpos[(size_t)grp0 * G + blk + 4].y : 0;
    } else {
        const int blk = lane >> 2;
        const int gg = (blk >= 8 && has1) ? grp0 + 1 : grp0;
        mir[0] = gpos[(size_t)gg * G + (blk & 7)].y;
        mir[1] = 0;
    }
    const PTask &Tk = tasks[t];
    const int np = __builtin_amdgcn_readfirstlane(Tk.np);
    const int shape = __builtin_amdgcn_readfirstlane(Tk.shape);
#define BBC_PAIR_CASE(SH, N) \
    case N: pair_dispatch_np<T, SH, N, NS, PIPE>(g0, g1, p0, p1, has1, Tk, lane, mir, set0); break;
    if (shape == 0) {
        switch (np) {
            BBC_PAIR_CASE(0, 1) BBC_PAIR_CASE(0, 2) BBC_PAIR_CASE(0, 3) BBC_PAIR_CASE(0, 4)
            BBC_PAIR_CASE(0, 5) BBC_PAIR_CASE(0, 6) BBC_PAIR_CASE(0, 7) BBC_PAIR_CASE(0, 8)
            default: break;
        }
    } else {
        switch (np) {
            BBC_PAIR_CASE(1, 1) BBC_PAIR_CASE(1, 2) BBC_PAIR_CASE(1, 3) BBC_PAIR_CASE(1, 4)
            default: break;
        }
    }
#undef BBC_PAIR_CASE
}

// Channel sums: Ct[ch][s][q] = sum_t w_t P[group][pair_t][s][slot], FP64
// accumulation in ascending pair order (stored as FP64, or in the FP32 form as
// float-float pairs for the compensated inverse transform).  One workgroup per momentum group reads
// the group's pair products pair by pair (pair-major entry lists) for up to
// kCombChunk channels; its 1024 lanes are 8 channel classes (ch mod 8) x 16
// spins x G momenta, and a lane keeps the sums of its class's (at most 8)
// channels in registers, the channel of each entry selected by a wave-uniform
// branch.  Every sum belongs to one lane and is formed in a fixed order (no
// atomics).  Entries are taken in batches of B whose loads are all issued
// first (the kernel is bound by the latency of these loads).
template <typename T, int B>
__global__ __launch_bounds__(1024) void k_pair_combine(const typename cplx_t<T>::type *__restrict__ P,
                                                       typename ct_t<T>::type *__restrict__ Ct, int ch0, int nch,
                                                       long V, const int2 *__restrict__ gpos, int gbase, int npair,
                                                       const CombEntry *__restrict__ comb,
                                                       const int32_t *__restrict__ comb_begin) {
    using T2 = typename cplx_t<T>::type;
    constexpr int G = GroupLayout<T2>::G;
    constexpr int NJ = kCombChunk / kCombSubs;      // channels per class
    static_assert(kCombSubs * 16 * G == 1024, "one lane per (class, spin, momentum)");
    const int grp = gbase + blockIdx.x;
    const int t = threadIdx.x;
    const int sub = __builtin_amdgcn_readfirstlane(t >> 7);
    const int s = (t >> 3) & 15, slot = t & 7;
    const T2 *pg = P + (size_t)grp * npair * 16 * G + s * G + slot;
    double2 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = double2{0.0, 0.0};
    const int eb = comb_begin[sub], ee = comb_begin[sub + 1];
    for (int i0 = eb; i0 < ee; i0 += B) {
        T2 v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = i0 + u < ee ? pg[(size_t)comb[i0 + u].pair * 16 * G] : T2{0, 0};
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (i0 + u >= ee) break;
            const int j = comb[i0 + u].ch >> 3;       // ch = sub + 8 j
            const double w = comb[i0 + u].w;
            switch (j) {
#define BBC_COMB_CASE(J) \
    case J: acc[J].x = fma(w, (double)v[u].x, acc[J].x); acc[J].y = fma(w, (double)v[u].y, acc[J].y); break;
                BBC_COMB_CASE(0) BBC_COMB_CASE(1) BBC_COMB_CASE(2) BBC_COMB_CASE(3)
                BBC_COMB_CASE(4) BBC_COMB_CASE(5) BBC_COMB_CASE(6) BBC_COMB_CASE(7)
#undef BBC_COMB_CASE
                default: break;
            }
        }
    }
    const int q = gpos[(size_t)grp * G + slot].x;
    if (q < 0) return;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int ch = sub + 8 * j;
        if (ch >= nch) continue;
        if constexpr (sizeof(T) == 4)        // FP32 form: the FP64 sums as float-float pairs
            Ct[((size_t)(ch0 + ch) * 16 + s) * V + q] = ffc{ff(acc[j].x), ff(acc[j].y)};
        else
            Ct[((size_t)(ch0 + ch) * 16 + s) * V + q] = T2{(T)acc[j].x, (T)acc[j].y};
    }
}

template <typename T, int NS, bool PIPE>
static void launch_pairs_v(const typename cplx_t<T>::type *Iq, typename cplx_t<T>::type *P, int nc,
                           const PairDevTables &tb, hipStream_t st) {
    constexpr int GPU_ = sizeof(T) == 8 ? 1 : 2;
    constexpr int PARTS = sizeof(T) == 8 ? 2 / NS : 1;
    const int nunit = (tb.ngroup + GPU_ - 1) / GPU_;
    const long nchunk = ((long)tb.ntask * PARTS + 3) / 4;
    if (nchunk == 0) return;
    // units per launch: below 2^32 work-items per dispatch
    const long max_wg = (1L << 32) / 256 - 64;
    const int per = (int)std::max<long>(8, std::min<long>(nunit, (max_wg / nchunk) / 8 * 8));
    for (int u0 = 0; u0 < nunit; u0 += per) {
        const int uc = std::min(per, nunit - u0);
        const long nwg = 8L * ((uc + 7) / 8) * nchunk;
        hipLaunchKernelGGL((k_pairs<T, NS, PIPE>), dim3((unsigned)nwg), dim3(256), 0, st, Iq, P, nc, u0, uc, tb.gpos,
                           tb.ngroup, tb.tasks, tb.ntask, tb.npair);
    }
}

template <typename T, bool PIPE, int KS = 2>
static void launch_pairs_lds(const typename cplx_t<T>::type *Iq, typename cplx_t<T>::type *P, int nc,
                             const PairDevTables &tb, hipStream_t st) {
    constexpr int GPU_ = sizeof(T) == 8 ? 1 : 2;
    const int nunit = (tb.ngroup + GPU_ - 1) / GPU_;
    const long nchunk = ((long)tb.ntask + 3) / 4;
    if (nchunk == 0) return;
    const long max_wg = (1L << 32) / 256 - 64;
    const int per = (int)std::max<long>(8, std::min<long>(nunit, (max_wg / nchunk) / 8 * 8));
    for (int u0 = 0; u0 < nunit; u0 += per) {
        const int uc = std::min(per, nunit - u0);
        const long nwg = 8L * ((uc + 7) / 8) * nchunk;
        hipLaunchKernelGGL((k_pairs_lds<T, PIPE, KS>), dim3((unsigned)nwg), dim3(256), 0, st, Iq, P, nc, u0, uc, tb.gpos,
                           tb.ngroup, tb.tasks, tb.ntask, tb.npair);
    }
}

template <bool PIPE>
static void launch_pairs_lds64s(const double2 *Iq, double2 *P, int nc, const PairDevTables &tb, hipStream_t st) {
    const int nunit = tb.ngroup;
    const long nchunk = ((long)tb.ntask * 2 + 3) / 4;
    if (nchunk == 0) return;
    const long max_wg = (1L << 32) / 256 - 64;
    const int per = (int)std::max<long>(8, std::min<long>(nunit, (max_wg / nchunk) / 8 * 8));
    for (int u0 = 0; u0 < nunit; u0 += per) {
        const int uc = std::min(per, nunit - u0);
        const long nwg = 8L * ((uc + 7) / 8) * nchunk;
        hipLaunchKernelGGL((k_pairs_lds64s<PIPE>), dim3((unsigned)nwg), dim3(256), 0, st, Iq, P, nc, u0, uc, tb.gpos,
                           tb.ngroup, tb.tasks, tb.ntask, tb.npair);
    }
}

static void launch_pairs_tiles64s(const double2 *Iq, double2 *P, int nc, const PairDevTables &tb, hipStream_t st) {
    const int nunit = tb.ngroup;
    const long nchunk = ((long)tb.ntile * 2 + 3) / 4;
    if (nchunk == 0) return;
    const long max_wg = (1L << 32) / 256 - 64;
    const int per = (int)std::max<long>(8, std::min<long>(nunit, (max_wg / nchunk) / 8 * 8));
    for (int u0 = 0; u0 < nunit; u0 += per) {
        const int uc = std::min(per, nunit - u0);
        const long nwg = 8L * ((uc + 7) / 8) * nchunk;
        hipLaunchKernelGGL(k_pairs_tiles64s, dim3((unsigned)nwg), dim3(256), 0, st, Iq, P, nc, u0, uc, tb.gpos,
                           tb.ngroup, tb.tiles, tb.ntile, tb.npair);
    }
}

static void launch_pairs_tiles32(const float2 *Iq, float2 *P, int nc, const PairDevTables &tb, hipStream_t st) {
    const int nunit = (tb.ngroup + 1) / 2;
    const long nchunk = ((long)tb.ntile + 3) / 4;
    if (nchunk == 0) return;
    const long max_wg = (1L << 32) / 256 - 64;
    const int per = (int)std::max<long>(8, std::min<long>(nunit, (max_wg / nchunk) / 8 * 8));
    for (int u0 = 0; u0 < nunit; u0 += per) {
        const int uc = std::min(per, nunit - u0);
        const long nwg = 8L * ((uc + 7) / 8) * nchunk;
        hipLaunchKernelGGL(k_pairs_tiles32, dim3((unsigned)nwg), dim3(256), 0, st, Iq, P, nc, u0, uc, tb.gpos,
                           tb.ngroup, tb.tiles, tb.ntile, tb.npair);
    }
}

// Variants (same products in the same order, so the same bits): FP64 0 = whole
// group per wave, 1 = whole group, pipelined, 2 = half group, 3 = half group,
// pipelined, 4 = operands staged through LDS, 5 = staged, double-buffered,
// 6 = staged per set of 4 momenta (half lines), 7 = the same, double-buffered,
// 8 = row tiles (three rows) staged per set of 4 momenta; FP32 0 = plain, 1 = pipelined, 2 = staged through LDS, 3 = staged,
// double-buffered, 4 = staged, 4 open indices per round, 5 = row tiles.
template <typename T>
void launch_pairs(const typename cplx_t<T>::type *Iq, typename cplx_t<T>::type *P, int nc, const PairDevTables &tb,
                  int variant, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        switch (variant) {
        case 1: launch_pairs_v<T, 2, true>(Iq, P, nc, tb, st); break;
        case 2: launch_pairs_v<T, 1, false>(Iq, P, nc, tb, st); break;
        case 3: launch_pairs_v<T, 1, true>(Iq, P, nc, tb, st); break;
        case 4: launch_pairs_lds<T, false>(Iq, P, nc, tb, st); break;
        case 5: launch_pairs_lds<T, true>(Iq, P, nc, tb, st); break;
        case 6: launch_pairs_lds64s<false>(Iq, P, nc, tb, st); break;
        case 7: launch_pairs_lds64s<true>(Iq, P, nc, tb, st); break;
        case 8: launch_pairs_tiles64s((const double2 *)Iq, (double2 *)P, nc, tb, st); break;
        default: launch_pairs_v<T, 2, false>(Iq, P, nc, tb, st); break;
        }
    } else {
        switch (variant) {
        case 1: launch_pairs_v<T, 2, true>(Iq, P, nc, tb, st); break;
        case 2: launch_pairs_lds<T, false>(Iq, P, nc, tb, st); break;
        case 3: launch_pairs_lds<T, true>(Iq, P, nc, tb, st); break;
        case 4: launch_pairs_lds<T, false, 4>(Iq, P, nc, tb, st); break;
        case 5: launch_pairs_tiles32((const float2 *)Iq, (float2 *)P, nc, tb, st); break;
        default: launch_pairs_v<T, 2, false>(Iq, P, nc, tb, st); break;
        }
    }
}

// Channel sums with the pair products staged through LDS: the workgroup of a
// momentum group copies PC consecutive pairs at a time (contiguous in P) into
// LDS with 16-byte lanes, then every lane applies its class's entries for those
// pairs from LDS, so each pair product is read from memory once per group (the
// classes of the direct form read a pair at different times, after it has left
// L2).  Lanes, sums and their order are those of k_pair_combine.  (Tried and
// slower: a second LDS buffer filled by direct loads while the first is used,
// and batches of LDS reads; both need registers that cost a workgroup per CU.)
template <typename T, int PC>
__global__ __launch_bounds__(1024) void k_pair_combine_lds(const typename cplx_t<T>::type *__restrict__ P,
                                                           typename ct_t<T>::type *__restrict__ Ct, int ch0,
                                                           int nch, long V, const int2 *__restrict__ gpos, int gbase,
                                                           int npair, const CombEntry *__restrict__ comb,
                                                           const int32_t *__restrict__ comb_begin) {
    using T2 = typename cplx_t<T>::type;
    constexpr int G = GroupLayout<T2>::G;
    constexpr int NJ = kCombChunk / kCombSubs;
    constexpr int PAIR16 = 16 * G * (int)sizeof(T2) / 16;      // 16-byte units per pair
    __shared__ float4 stage[PC * PAIR16];
    const int grp = gbase + blockIdx.x;
    const int t = threadIdx.x;
    const int sub = __builtin_amdgcn_readfirstlane(t >> 7);
    const int s = (t >> 3) & 15, slot = t & 7;
    const float4 *pg4 = (const float4 *)(P + (size_t)grp * npair * 16 * G);
    const T2 *st2 = (const T2 *)stage + s * G + slot;
    double2 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = double2{0.0, 0.0};
    int e = comb_begin[sub];
    const int ee = comb_begin[sub + 1];
    // the class's current entry (whole 16-byte record: pair, ch, w), carried across chunks
    int4 cur = e < ee ? *(const int4 *)&comb[e] : int4{npair, 0, 0, 0};
    for (int p0 = 0; p0 < npair; p0 += PC) {
        const int np = min(PC, npair - p0);
        __syncthreads();                                           // previous chunk consumed
        for (int i = t; i < np * PAIR16; i += 1024) stage[i] = pg4[(size_t)p0 * PAIR16 + i];
        __syncthreads();
        // this class's entries with pairs in [p0, p0 + np), in ascending pair order; the
        // next record is requested together with the current entry's operand
        while (cur.x < p0 + np) {
            const int4 nxt = e + 1 < ee ? *(const int4 *)&comb[e + 1] : int4{npair, 0, 0, 0};
            const T2 v = st2[(size_t)(cur.x - p0) * 16 * G];
            const double w = __hiloint2double(cur.w, cur.z);
            switch (cur.y >> 3) {
#define BBC_COMB_CASE(J) \
    case J: acc[J].x = fma(w, (double)v.x, acc[J].x); acc[J].y = fma(w, (double)v.y, acc[J].y); break;
                BBC_COMB_CASE(0) BBC_COMB_CASE(1) BBC_COMB_CASE(2) BBC_COMB_CASE(3)
                BBC_COMB_CASE(4) BBC_COMB_CASE(5) BBC_COMB_CASE(6) BBC_COMB_CASE(7)
#undef BBC_COMB_CASE
                default: break;
            }
            cur = nxt;
            ++e;
        }
    }
    const int q = gpos[(size_t)grp * G + slot].x;
    if (q < 0) return;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int ch = sub + 8 * j;
        if (ch >= nch) continue;
        if constexpr (sizeof(T) == 4)
            Ct[((size_t)(ch0 + ch) * 16 + s) * V + q] = ffc{ff(acc[j].x), ff(acc[j].y)};
        else
            Ct[((size_t)(ch0 + ch) * 16 + s) * V + q] = T2{(T)acc[j].x, (T)acc[j].y};
    }
}

// Variants (same sums in the same order): entries per load batch, 0 = 8, 1 = 16;
// 2 = pair products staged through LDS, 64 KB at a time (FP64 32 pairs, FP32 64).
template <typename T>
void launch_pair_combine(const typename cplx_t<T>::type *P, typename ct_t<T>::type *Ct, int n_ch, long V,
                         const PairDevTables &tb, int variant, hipStream_t st) {
    const long max_wg = (1L << 32) / 1024 - 64;
    for (int c0 = 0; c0 < n_ch; c0 += kCombChunk) {
        const int nch = std::min(kCombChunk, n_ch - c0);
        const int32_t *cb = tb.comb_begin + (size_t)(c0 / kCombChunk) * kCombSubs;
        for (long g0 = 0; g0 < tb.ngroup; g0 += max_wg) {
            const long gc = std::min<long>(max_wg, tb.ngroup - g0);
            if (variant == 2)
                hipLaunchKernelGGL((k_pair_combine_lds<T, sizeof(T) == 4 ? 64 : 32>), dim3((unsigned)gc), dim3(1024), 0,
                                   st, P, Ct, c0, nch, V, tb.gpos, (int)g0, tb.npair, tb.comb, cb);
            else if (variant == 1)
                hipLaunchKernelGGL((k_pair_combine<T, 16>), dim3((unsigned)gc), dim3(1024), 0, st, P, Ct, c0, nch, V,
                                   tb.gpos, (int)g0, tb.npair, tb.comb, cb);
            else
                hipLaunchKernelGGL((k_pair_combine<T, 8>), dim3((unsigned)gc), dim3(1024), 0, st, P, Ct, c0, nch, V,
                                   tb.gpos, (int)g0, tb.npair, tb.comb, cb);
        }
    }
}

// ----------------------------------------------------------------------------
// Finalisation: C(r) = (1/V) sum_q ... is already summed by the inverse FFT;
// multiply by exp(E_ch (t - t0)) / V (Sec. 2 Eq. (2)) and write [r][spin].
// With scale_out (FP32 form) the FP64 factor is written there instead and the
// field keeps only 1/V.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(const typename ct_t<T>::type *__restrict__ Ct,
                                                  typename cplx_t<T>::type *__restrict__ out, int n_ch, int V,
                                                  const double *__restrict__ energy, double dt, double inv_v,
                                                  double *__restrict__ scale_out, const uint32_t *__restrict__ kmax,
                                                  const int2 *__restrict__ content, const SliceArgs *__restrict__ ia,
                                                  int full) {
    using T2 = typename cplx_t<T>::type;
    using TC = typename ct_t<T>::type;
    if (ia) {
        out = (T2 *)ia->out;
        scale_out = ia->scale;
        dt = ia->dt;
    }
    // a tile of 256 sites x 16 spins of one channel: read along the sites (one spin
    // row at a time), written as one contiguous run of the [site][spin] output
    __shared__ TC tile[256][17];
    const int t = threadIdx.x;
    const long nchunk = (V + 255) / 256;
    for (long blk = blockIdx.x; blk < (long)n_ch * nchunk; blk += gridDim.x) {
        const int m = (int)(blk / nchunk);
        const int x0 = (int)(blk - (long)m * nchunk) * 256;
        const double e = energy ? exp(energy[m] * dt) : 1.0;
        T f;
        if (scale_out) {
            // FP64 factor: exp(E (t - t0)) and the inverse of the propagator rescale,
            // kappa_l^-n_l kappa_s^-n_s with kappa = 2^-e (exact powers of two)
            f = T(inv_v);
            if (x0 == 0 && t == 0) {
                const int el = kmax ? pow2_exponent(__uint_as_float(kmax[0])) : 0;
                const int es = kmax ? pow2_exponent(__uint_as_float(kmax[1])) : 0;
                const int2 nls = content[m];
                scale_out[m] = ldexp(e, el * nls.x + es * nls.y);
            }
        } else {
            f = T(e * inv_v);
        }
        const int x = x0 + t;
        if (x < V) {
#pragma unroll
            for (int s = 0; s < 16; ++s) tile[t][s] = Ct[((size_t)m * 16 + s) * V + x];
        }
        __syncthreads();
        const int nsite = min(256, V - x0);
        // all-components request: this evaluation's 16 values go to alpha = 2 h1 + a,
        // beta = 2 h2 + b, ... of the 256-value site record (h = the lower-pair bits)
        const int ostride = full >= 0 ? 256 : 16;
        const int obase = full >= 0 ? 2 * (full & 1) + 8 * ((full >> 1) & 1) + 32 * ((full >> 2) & 1) +
                                          128 * ((full >> 3) & 1)
                                    : 0;
        T2 *o = out + ((size_t)m * V + x0) * ostride;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int idx = k * 256 + t, site = idx >> 4, s = idx & 15;
            if (site < nsite) {
                const TC v = tile[site][s];
                const int oi = full >= 0 ? site * 256 + obase + (s & 1) + 4 * ((s >> 1) & 1) + 16 * ((s >> 2) & 1) +
                                               64 * ((s >> 3) & 1)
                                         : idx;
                if constexpr (sizeof(T) == 4)    // float-float: one rounding of hi + lo, times 1/V
                    o[oi] = T2{(T)(((double)v.x.hi + (double)v.x.lo) * (double)f),
                               (T)(((double)v.y.hi + (double)v.y.lo) * (double)f)};
                else
                    o[oi] = T2{v.x * f, v.y * f};
            }
        }
        __syncthreads();
    }
}

template <typename T>
void launch_finalize(const typename ct_t<T>::type *Ct, typename cplx_t<T>::type *out, int n_ch, int V,
                     const double *energy, double dt, double inv_v, double *scale_out, const uint32_t *kmax,
                     const int2 *content, hipStream_t st, const SliceArgs *ia, int full) {
    const long nblk = (long)n_ch * ((V + 255) / 256);
    const unsigned grid = (unsigned)std::min<long>(nblk, 1L << 22);
    hipLaunchKernelGGL((k_finalize<T>), dim3(grid), dim3(256), 0, st, Ct, out, n_ch, V, energy, dt, inv_v,
                       scale_out, kmax, content, ia, full);
}

// explicit instantiations
template void launch_blocks<double>(const double2 *, const double2 *, double2 *, int, int, int, const BlockComp *,
                                    const uint32_t *, const BlockPatterns &, const uint32_t *, int, hipStream_t,
                                    const SliceArgs *);
template void launch_blocks<float>(const float2 *, const float2 *, float2 *, int, int, int, const BlockComp *,
                                   const uint32_t *, const BlockPatterns &, const uint32_t *, int, hipStream_t,
                                   const SliceArgs *);
template int launch_fft3d<double>(double2 *, long, const int[3], int, hipStream_t);
template int launch_fft3d_zgrouped<double>(double2 *, double2 *, int, const int[3], const int *, const int *, int,
                                            hipStream_t);
template int launch_fft3d_zgrouped<float>(float2 *, float2 *, int, const int[3], const int *, const int *, int,
                                           hipStream_t);
template bool fft3d_zgrouped_fits<double>(const int[3]);
template bool fft3d_onepass_fits<double>(const int[3]);
template bool fft3d_onepass_fits<float>(const int[3]);
template int launch_fft3d_onepass<double>(const double2 *, double2 *, int, const int[3], const int *, hipStream_t);
template int launch_fft3d_onepass<float>(const float2 *, float2 *, int, const int[3], const int *, hipStream_t);
template bool fft3d_zgrouped_fits<float>(const int[3]);
template int launch_fft3d<float>(float2 *, long, const int[3], int, hipStream_t);
template int launch_fft3d<ff>(ffc *, long, const int[3], int, hipStream_t);
template void launch_transpose_grouped<double>(const double2 *, double2 *, int, long, int, const int2 *,
                                               hipStream_t);
template void launch_transpose_grouped<float>(const float2 *, float2 *, int, long, int, const int2 *, hipStream_t);
template bool fft3d_grouped_fits<double>(const int[3]);
template bool fft3d_grouped_fits<float>(const int[3]);
template int launch_fft3d_grouped<double>(const double2 *, double2 *, int, const int[3], int, const int2 *,
                                          hipStream_t);
template int launch_fft3d_grouped<float>(const float2 *, float2 *, int, const int[3], int, const int2 *, hipStream_t);
template void launch_pairs<double>(const double2 *, double2 *, int, const PairDevTables &, int, hipStream_t);
template void launch_pairs<float>(const float2 *, float2 *, int, const PairDevTables &, int, hipStream_t);
template void launch_pair_combine<double>(const double2 *, double2 *, int, long, const PairDevTables &, int,
                                          hipStream_t);
template void launch_pair_combine<float>(const float2 *, ffc *, int, long, const PairDevTables &, int,
                                         hipStream_t);
template void launch_finalize<double>(const double2 *, double2 *, int, int, const double *, double, double,
                                      double *, const uint32_t *, const int2 *, hipStream_t, const SliceArgs *, int);
template void launch_finalize<float>(const ffc *, float2 *, int, int, const double *, double, double, double *,
                                     const uint32_t *, const int2 *, hipStream_t, const SliceArgs *, int);

}  // namespace bbc
