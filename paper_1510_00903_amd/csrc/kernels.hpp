// gfx950 kernels of the effective block algorithm (declarations shared by the
// host driver).  Paper: arXiv:1510.00903, Sec. 3.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pairs.hpp"

namespace bbc {

// Device pointers of the pair tables of one plan (pairs.hpp).
struct PairDevTables {
    const int2 *gpos;             // per grouped position: (momentum or -1, lane of -q in the group)
    int ngroup;                   // momentum groups (G positions each)
    const PTask *tasks;
    int ntask;
    const PTask *tiles;           // the same products as row tiles (pairs.hpp)
    int ntile;
    int npair;
    const CombEntry *comb;        // channel terms, pair-major (pairs.hpp)
    const int32_t *comb_begin;    // per chunk of kCombChunk channels and class: entry ranges
};

// Blocks of 256 threads for a one-dimensional launch over n items, capped so
// that a dispatch stays below 2^32 work-items (the packet's grid size is 32-bit);
// such kernels loop over their items with the grid stride.
inline unsigned grid1d(long n) {
    const long b = (n + 255) / 256;
    return (unsigned)(b < (1L << 22) ? (b > 0 ? b : 1) : (1L << 22));
}

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };

// Float-float real: the value hi + lo with |lo| <= ulp(hi) / 2 (about 48
// significant bits from FP32 arithmetic).  The FP32 form sums the channels in
// FP64 and keeps them as float-float pairs, and the inverse transform (the sum
// over momenta that gives C(r)) runs in compensated float-float arithmetic
// (error-free TwoSum / FMA TwoProd steps, kernels.hip); the field is rounded
// to FP32 once, when it is written out.
struct ff {
    float hi, lo;
    ff() = default;
    __host__ __device__ constexpr ff(float h, float l) : hi(h), lo(l) {}
    __host__ __device__ explicit ff(double d) : hi((float)d), lo((float)(d - (double)(float)d)) {}
};
struct ffc {
    ff x, y;
};
template <> struct cplx_t<ff> { using type = ffc; };
// Type of the contracted field Ct (channel sums, then the inverse transform):
// FP64 form double2, FP32 form float-float pairs.
template <typename T> struct ct_t { using type = typename cplx_t<T>::type; };
template <> struct ct_t<float> { using type = ffc; };
template <typename T> struct ct_real { using type = T; };
template <> struct ct_real<float> { using type = ff; };

// Component patterns of the block kernel: components [begin, end) share the
// flavours of roles a, b, c (0 light, 1 strange) and the spin structure, given
// as monomial matrices Gamma_1(mu, p1[mu]) = i^k1[mu], Gamma_2(g, p2[g]) = i^k2[g].
// new_diquark: the diquark tensor (qa, qb, Gamma_1) differs from the previous pattern's.
struct BlockPattern {
    int begin, end;
    uint8_t qa, qb, qc, new_diquark;
    uint8_t p1[4], k1[4], p2[4], k2[4];
};
constexpr int kMaxBlockPatterns = 40;
struct BlockPatterns {
    int n;
    int any_imag;         // some term has the factor-i bit
    BlockPattern p[kMaxBlockPatterns];
};

// Arguments of one time slice that change from slice to slice: the two
// propagator slices, the output slab, the FP32 scale row (else NULL) and t - t0.
// Where a launcher takes `ia` (a device copy of this record), a non-NULL `ia`
// replaces the pointers and dt it is given, so that one captured kernel
// sequence serves every slice of a request shape (graph replay in the serving
// loop): launch_slice_args writes the next slice's record, stream-ordered.
struct SliceArgs {
    const void *sl, *ss;
    void *out;
    double *scale;
    double dt;
};
void launch_slice_args(SliceArgs *dst, const SliceArgs &v, hipStream_t st);

// One block component: its number of terms n, its first two terms t0, t1 (0 where
// absent), and the index in the term array of its third term.  A term is
// ab | ec << 8 | sign << 12 | i << 13, with ab = 12 ea + eb the diquark column and
// ec the third propagator's column (term value: sign * i^bit13 * sum_c
// Q[c][ea][eb] S_c[row + c][ec]).  Records let a thread fetch the next
// component with one load while it works on the current one.
struct BlockComp {
    uint32_t t0, t1, rest, n;
};

template <typename T>
void launch_blocks(const typename cplx_t<T>::type *Sl, const typename cplx_t<T>::type *Ss,
                   typename cplx_t<T>::type *I, int V, int nc, int g0, const BlockComp *comps,
                   const uint32_t *terms, const BlockPatterns &pt, const uint32_t *kmax, int variant,
                   hipStream_t st, const SliceArgs *ia = nullptr);

// Kernel variants of one request shape (every variant forms the same values in
// the same order, so the results are the same bits; only speed differs):
//   pairs  - pair-product kernel: FP64 0 = whole group per wave, 1 = pipelined,
//            2 = half group per wave, 3 = half group, pipelined, 4 = operands staged
//            through LDS, 5 = staged, double-buffered, 6 = staged per set of 4 momenta,
//            7 = the same, double-buffered; FP32 0, 1 = pipelined,
//            2 = staged through LDS, 3 = staged, double-buffered, 4 = staged, 4 open
//            indices per round;
//   blocks - block kernel sites per workgroup x component shares: 0 = 4x2, 1 = 4x4, 2 = 8x2;
//   planes - plane-pass FFT planes per workgroup: 0 = as many as 80 KB of LDS hold, 1 = half;
//   slices - time slices of one request run at once (1 << slices), each on its own
//            stream and workspace;
//   combine - channel sums: entries per load batch, 0 = 8, 1 = 16; 2 = pair products staged
//            through LDS (read once per group).
struct Tuning {
    int pairs = 0, blocks = 0, planes = 0, slices = 0, combine = 0;
};
constexpr int kPairVariants64 = 9, kPairVariants32 = 6, kBlockVariants = 3, kPlaneVariants = 2, kSliceVariants = 4,
              kCombineVariants = 3;
constexpr int kMaxSliceStreams = 1 << (kSliceVariants - 1);

// FP32 form: per-flavour max |Re|,|Im| of a slice into kmax[0] (light), kmax[1] (strange).
void launch_absmax(const float2 *Sl, const float2 *Ss, long n, uint32_t *kmax, hipStream_t st,
                   const SliceArgs *ia = nullptr);

template <typename T>
int launch_fft3d(typename cplx_t<T>::type *data, long ncomp, const int L[3], int sign, hipStream_t st);
// Forward FFT of the 2 nc intermediates (in place in `in` for x and y) with the z
// pass writing straight into the momentum groups of `out`; posof[q] = position
// of momentum q; xrun (run-ordered groups, else NULL) = first group of each
// x-row's run.  Returns kernels launched, -1 if the lattice does not fit.
template <typename T> bool fft3d_zgrouped_fits(const int L[3]);
template <typename T>
int launch_fft3d_zgrouped(typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                          const int *posof, const int *xrun, int plane_variant, hipStream_t st);

// One-pass forward FFT into the run-ordered groups (FP32, cubic 24 or 32):
// -1 where it does not apply.
template <typename T> bool fft3d_onepass_fits(const int L[3]);
template <typename T>
int launch_fft3d_onepass(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                         const int *xrun, hipStream_t st);

// Momentum-grouped copy: in [g][nc][V] (component-major) -> out, per group of G
// = 8 momenta and component, the G momenta and both sink spins ([c][G][g]);
// gpos is the position table of the groups.
template <typename T>
void launch_transpose_grouped(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, long V,
                              int ngroup, const int2 *gpos, hipStream_t st);

// Forward 3-D FFT fused with the grouped copy (one pass), for cubic lattices
// whose N^3 complex values fit in 64 KB; returns -1 where it does not apply.
template <typename T> bool fft3d_grouped_fits(const int L[3]);
template <typename T>
int launch_fft3d_grouped(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, int nc, const int L[3],
                         int ngroup, const int2 *gpos, hipStream_t st);

// Pair products P[group][pair][spin][G] of every task (MFMA), then the channel
// sums Ct[ch][spin][q] = sum_t w_t P[pair_t] (ascending pair order, FP64 accumulation).
template <typename T>
void launch_pairs(const typename cplx_t<T>::type *Iq, typename cplx_t<T>::type *P, int nc,
                  const PairDevTables &tb, int variant, hipStream_t st);
template <typename T>
void launch_pair_combine(const typename cplx_t<T>::type *P, typename ct_t<T>::type *Ct, int n_ch, long V,
                         const PairDevTables &tb, int variant, hipStream_t st);

template <typename T>
void launch_finalize(const typename ct_t<T>::type *Ct, typename cplx_t<T>::type *out, int n_ch, int V,
                     const double *energy, double dt, double inv_v, double *scale_out, const uint32_t *kmax,
                     const int2 *content, hipStream_t st, const SliceArgs *ia = nullptr, int full = -1);

bool fft_size_supported(int n);

// Post-processing of C(r, t) (Sec. 2).
struct SpinWeights4 {            // up to 4 output combinations of the 16 spin values
    double2 w[4][16];
    int n;
};
template <typename T>
void launch_spin_project(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, long nsite, int n_out,
                         const double *W, hipStream_t st);
template <typename T>
void launch_cubic_project(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, long n_fields, int L,
                          int n_comp, int complement, hipStream_t st);
void launch_central_potential(const double2 *R, double2 *Vout, const int L[3], long n_fields, int n_t,
                              double inv_2mu, hipStream_t st);
// Forward/backward (CPT) average of Sec. 6, in place on R.
template <typename T>
void launch_cpt_average(typename cplx_t<T>::type *R, const typename cplx_t<T>::type *B, long per_ch, int n_ch,
                        double sign, const double *sf, const double *sb, double *scale_out, hipStream_t st);

}  // namespace bbc
