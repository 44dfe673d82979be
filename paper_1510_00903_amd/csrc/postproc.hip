// gfx950 kernels for the post-processing of C(r, t) (Sec. 2): projection of the
// spin values to total spin (J, M), projection of the relative coordinate onto
// the A1+ representation of the cubic group, and the leading-order central
// potential of the HAL QCD method.  Paper: arXiv:1510.00903, Sec. 2.
#include "kernels.hpp"

namespace bbc {

// ----------------------------------------------------------------------------
// Post-processing of C(r, t) (Sec. 2): spin projection, projection of the
// spatial argument onto the A1+ representation of the cubic group, and the
// leading-order central potential.  All three are site-local or stencil work
// on the output field, bound by HBM.
// ----------------------------------------------------------------------------
// Spin projection: out[f][r][m0 + m] = sum_s W.w[m][s] in[f][r][s], m < W.n (<= 4
// outputs per launch; the weights travel in the kernel arguments).  One thread per site.
template <typename T>
__global__ __launch_bounds__(256) void k_spin_project(const typename cplx_t<T>::type *__restrict__ in,
                                                      typename cplx_t<T>::type *__restrict__ out, long nsite,
                                                      int n_out, int m0, SpinWeights4 W) {
    using T2 = typename cplx_t<T>::type;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nsite; i += (long)gridDim.x * blockDim.x) {
    const T2 *p = in + i * 16;
    double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const T2 v = p[s];
        const double vx = v.x, vy = v.y;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double2 w = W.w[m][s];
            acc[m].x += w.x * vx - w.y * vy;
            acc[m].y += w.x * vy + w.y * vx;
        }
    }
    T2 *q = out + i * n_out + m0;
    for (int m = 0; m < W.n; ++m) q[m] = T2{T(acc[m].x), T(acc[m].y)};
    }
}

// The 24 proper rotations of the cube as signed permutations of (x, y, z):
// r'_d = s[d] * r_{p[d]}, enumerated at compile time (permutation parity times
// the product of the signs must be +1).
struct CubeRot {
    int p[3], s[3];
};
struct CubeRotTable {
    CubeRot r[24];
};
constexpr CubeRotTable make_cube_rotations() {
    CubeRotTable t{};
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int k = 0;
    for (int i = 0; i < 6; ++i) {
        const int inv = (perms[i][0] > perms[i][1]) + (perms[i][0] > perms[i][2]) + (perms[i][1] > perms[i][2]);
        for (int sg = 0; sg < 8; ++sg) {
            const int s0 = (sg & 1) ? -1 : 1, s1 = (sg & 2) ? -1 : 1, s2 = (sg & 4) ? -1 : 1;
            if (((inv & 1) ? -1 : 1) * s0 * s1 * s2 != 1) continue;
            t.r[k].p[0] = perms[i][0]; t.r[k].p[1] = perms[i][1]; t.r[k].p[2] = perms[i][2];
            t.r[k].s[0] = s0; t.r[k].s[1] = s1; t.r[k].s[2] = s2;
            ++k;
        }
    }
    return t;
}
constexpr CubeRotTable kCubeRot = make_cube_rotations();

// Sum over the 24 rotations of v(R r): r and -r (mod L) per axis are formed once.
template <typename Load>
__device__ __forceinline__ double2 cube_sum(const int r[3], int L, Load load) {
    int pos[3], neg[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos[d] = r[d];
        neg[d] = r[d] == 0 ? 0 : L - r[d];
    }
    double ax = 0, ay = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        const CubeRot &R = kCubeRot.r[k];
        const int x = R.s[0] > 0 ? pos[R.p[0]] : neg[R.p[0]];
        const int y = R.s[1] > 0 ? pos[R.p[1]] : neg[R.p[1]];
        const int z = R.s[2] > 0 ? pos[R.p[2]] : neg[R.p[2]];
        const auto v = load((z * L + y) * L + x);
        ax += v.x;
        ay += v.y;
    }
    return double2{ax, ay};
}

// A1+ projection over the 24 proper rotations of the cube: thread = (field,
// site, component), the rotated values gathered from global memory (L2).
template <typename T>
__global__ __launch_bounds__(256) void k_cubic_project(const typename cplx_t<T>::type *__restrict__ in,
                                                       typename cplx_t<T>::type *__restrict__ out, long n_fields,
                                                       int L, int n_comp, int complement) {
    using T2 = typename cplx_t<T>::type;
    const long V = (long)L * L * L;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_fields * V * n_comp;
         i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % n_comp);
    const long site = (i / n_comp) % V;
    const long f = i / (n_comp * V);
    const int si = (int)site, r[3] = {si % L, (si / L) % L, si / (L * L)};
    const T2 *src = in + f * V * n_comp + c;
    double2 a = cube_sum(r, L, [&](int s) { return src[(long)s * n_comp]; });
    a.x *= 1.0 / 24.0;
    a.y *= 1.0 / 24.0;
    if (complement) {
        const T2 v = src[site * n_comp];
        a.x = v.x - a.x;
        a.y = v.y - a.y;
    }
    out[i] = T2{T(a.x), T(a.y)};
    }
}

// The same projection with one component of one field staged whole in LDS
// (lattices with L^3 complex values <= 64 KB): one workgroup per (field,
// component), placed XCD-aware so that the components of a field share an L2;
// the 24 rotated reads per output come from LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_cubic_project_lds(const typename cplx_t<T>::type *__restrict__ in,
                                                           typename cplx_t<T>::type *__restrict__ out, long n_fields,
                                                           int L, int n_comp, int complement) {
    using T2 = typename cplx_t<T>::type;
    extern __shared__ unsigned char lds_raw[];
    T2 *buf = reinterpret_cast<T2 *>(lds_raw);
    const long V = (long)L * L * L;
    const long nwg = n_fields * n_comp;
    const long P8 = (nwg + 7) / 8;
    const long id = (blockIdx.x & 7) * P8 + (blockIdx.x >> 3);
    if (id >= nwg) return;
    const long f = id / n_comp;
    const int c = (int)(id - f * n_comp);
    const T2 *src = in + f * V * n_comp + c;
    const int Vi = (int)V;
    for (int s = threadIdx.x; s < Vi; s += 256) buf[s] = src[(long)s * n_comp];
    __syncthreads();
    T2 *dst = out + f * V * n_comp + c;
    for (int s = threadIdx.x; s < Vi; s += 256) {
        const int r[3] = {s % L, (s / L) % L, s / (L * L)};
        double2 a = cube_sum(r, L, [&](int q) { return buf[q]; });
        a.x *= 1.0 / 24.0;
        a.y *= 1.0 / 24.0;
        if (complement) {
            const T2 v = buf[s];
            a.x = v.x - a.x;
            a.y = v.y - a.y;
        }
        dst[(long)s * n_comp] = T2{T(a.x), T(a.y)};
    }
}

// Central potential at slice t of n_t consecutive slices (t = 1 .. n_t - 2) of
// each of n_fields independent sequences R[f][t][site]:
//   V = (lap R(t) * inv_2mu - (R(t+1) - R(t-1)) / 2) / R(t), six-point periodic Laplacian.
__global__ __launch_bounds__(256) void k_central_potential(const double2 *__restrict__ R, double2 *__restrict__ Vout,
                                                           int Lx, int Ly, int Lz, long n_fields, int n_t,
                                                           double inv_2mu) {
    const long V = (long)Lx * Ly * Lz;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_fields * (n_t - 2) * V;
         i += (long)gridDim.x * blockDim.x) {
    const long site = i % V;
    const long ft = i / V;                         // f * (n_t - 2) + (t - 1)
    const long f = ft / (n_t - 2);
    const int t = (int)(ft - f * (n_t - 2)) + 1;
    const int x = (int)(site % Lx), y = (int)((site / Lx) % Ly), z = (int)(site / ((long)Lx * Ly));
    const double2 *Rf = R + f * n_t * V;
    const double2 *Rt = Rf + (long)t * V;
    auto at = [&](int xx, int yy, int zz) { return Rt[((long)zz * Ly + yy) * Lx + xx]; };
    const double2 c = Rt[site];
    const double2 n[6] = {at((x + 1) % Lx, y, z), at((x + Lx - 1) % Lx, y, z), at(x, (y + 1) % Ly, z),
                          at(x, (y + Ly - 1) % Ly, z), at(x, y, (z + 1) % Lz), at(x, y, (z + Lz - 1) % Lz)};
    double lx = -6.0 * c.x, ly = -6.0 * c.y;
#pragma unroll
    for (int k = 0; k < 6; ++k) { lx += n[k].x; ly += n[k].y; }
    const double2 up = Rf[(long)(t + 1) * V + site], dn = Rf[(long)(t - 1) * V + site];
    const double nx = lx * inv_2mu - 0.5 * (up.x - dn.x);
    const double ny = ly * inv_2mu - 0.5 * (up.y - dn.y);
    const double den = c.x * c.x + c.y * c.y;     // (nx + i ny) / (c.x + i c.y)
    Vout[i] = double2{(nx * c.x + ny * c.y) / den, (ny * c.x - nx * c.y) / den};
    }
}

// ----------------------------------------------------------------------------
// Forward/backward (CPT) average (Sec. 6): R = a C_fwd + b C_bwd elementwise
// over n_ch fields of per_ch values, R overwriting C_fwd.  FP64: a = 1/2,
// b = sign/2.  FP32: each part carries its own per-channel scale (sf, sb); the
// result is stored against m = max(sf, sb) with a = sf / (2 m), b = sign sb / (2 m),
// computed in FP64 and rounded once, and m is written to scale_out (a buffer
// distinct from sf and sb).
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_cpt_average(typename cplx_t<T>::type *__restrict__ R,
                                                     const typename cplx_t<T>::type *__restrict__ B, long per_ch,
                                                     int n_ch, double sign, const double *__restrict__ sf,
                                                     const double *__restrict__ sb, double *__restrict__ scale_out) {
    using T2 = typename cplx_t<T>::type;
    const long n = per_ch * n_ch;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double a = 0.5, b = 0.5 * sign;
        if (sf) {
            const int ch = (int)(i / per_ch);
            const double f = sf[ch], g = sb[ch], m = fmax(f, g);
            a *= f / m;
            b *= g / m;
            if (i - (long)ch * per_ch == 0) scale_out[ch] = m;
        }
        const T2 x = R[i], y = B[i];
        R[i] = T2{T(a * (double)x.x + b * (double)y.x), T(a * (double)x.y + b * (double)y.y)};
    }
}

template <typename T>
void launch_spin_project(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, long nsite, int n_out,
                         const double *W, hipStream_t st) {
    for (int m0 = 0; m0 < n_out; m0 += 4) {
        SpinWeights4 w{};
        w.n = n_out - m0 < 4 ? n_out - m0 : 4;
        for (int m = 0; m < w.n; ++m)
            for (int s = 0; s < 16; ++s) w.w[m][s] = double2{W[((m0 + m) * 16 + s) * 2], W[((m0 + m) * 16 + s) * 2 + 1]};
        hipLaunchKernelGGL((k_spin_project<T>), dim3(grid1d(nsite)), dim3(256), 0, st, in, out,
                           nsite, n_out, m0, w);
    }
}

template <typename T>
void launch_cubic_project(const typename cplx_t<T>::type *in, typename cplx_t<T>::type *out, long n_fields, int L,
                          int n_comp, int complement, hipStream_t st) {
    using T2 = typename cplx_t<T>::type;
    const long V = (long)L * L * L;
    if (V * (long)sizeof(T2) <= 65536 && n_fields * n_comp < (1L << 24) - 8) {
        const long nwg = n_fields * n_comp;
        hipLaunchKernelGGL((k_cubic_project_lds<T>), dim3((unsigned)(8 * ((nwg + 7) / 8))), dim3(256),
                           V * sizeof(T2), st, in, out, n_fields, L, n_comp, complement);
        return;
    }
    const long n = n_fields * V * n_comp;
    hipLaunchKernelGGL((k_cubic_project<T>), dim3(grid1d(n)), dim3(256), 0, st, in, out, n_fields,
                       L, n_comp, complement);
}

void launch_central_potential(const double2 *R, double2 *Vout, const int L[3], long n_fields, int n_t,
                              double inv_2mu, hipStream_t st) {
    const long n = n_fields * (n_t - 2) * L[0] * L[1] * L[2];
    hipLaunchKernelGGL(k_central_potential, dim3(grid1d(n)), dim3(256), 0, st, R, Vout, L[0], L[1],
                       L[2], n_fields, n_t, inv_2mu);
}

template <typename T>
void launch_cpt_average(typename cplx_t<T>::type *R, const typename cplx_t<T>::type *B, long per_ch, int n_ch,
                        double sign, const double *sf, const double *sb, double *scale_out, hipStream_t st) {
    const long n = per_ch * n_ch;
    hipLaunchKernelGGL((k_cpt_average<T>), dim3(grid1d(n)), dim3(256), 0, st, R, B, per_ch, n_ch, sign, sf, sb,
                       scale_out);
}

// explicit instantiations
template void launch_spin_project<double>(const double2 *, double2 *, long, int, const double *, hipStream_t);
template void launch_spin_project<float>(const float2 *, float2 *, long, int, const double *, hipStream_t);
template void launch_cubic_project<double>(const double2 *, double2 *, long, int, int, int, hipStream_t);
template void launch_cubic_project<float>(const float2 *, float2 *, long, int, int, int, hipStream_t);
template void launch_cpt_average<double>(double2 *, const double2 *, long, int, double, const double *,
                                         const double *, double *, hipStream_t);
template void launch_cpt_average<float>(float2 *, const float2 *, long, int, double, const double *, const double *,
                                        double *, hipStream_t);

}  // namespace bbc
