// The paper's own route to the spectral function of the free response
// (Section 8.A eq. sf-of-response-time): the electronic densities of Section 5
// split into empty (rho^+) and occupied (rhobar^-(s) = rho^-(-s)) parts on the
// mesh, their Fourier transforms to time, the local product
//   a_{mu nu}(t) = 2 V_mu^{ab} rho^+_{bc}(t) V_nu^{cd} rhobar^-_{da}(t)
// time by time, and the transform back to the mesh.  On the mesh the two
// transforms are discrete Fourier sums of length L, the length of the linear
// convolution (so the cyclic one has no wrap-around); both are done as FP64
// MFMA GEMMs with explicit cosine/sine matrices, which take any L, since only
// L/2 + 1 time points are needed (real spectra) and the matrices are small.
#include "gw_internal.h"
#include "gw_prof.h"

#include <algorithm>

namespace gwk {
namespace {

// rho[k][a][b] = sum over the levels i of bin k of (1 - phi_i) X_a^i X_b^i
//             + sum over the levels of bin k - 1 of phi_i X_a^i X_b^i.
// Levels are listed bin by bin: lev[start[k] .. start[k+1]) have bin k.
__global__ __launch_bounds__(256) void k_rho_bins(int n_orb, const double *__restrict__ X,
                                                  const int32_t *__restrict__ lev, const double *__restrict__ ph,
                                                  const int32_t *__restrict__ start, double *__restrict__ rho) {
    const int k = blockIdx.y;
    const int64_t nn = (int64_t)n_orb * n_orb;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const int a = (int)(e / n_orb), b = (int)(e % n_orb);
    const double *xa = X + (int64_t)a * n_orb;
    const double *xb = X + (int64_t)b * n_orb;
    double acc = 0.0;
    for (int i = start[k]; i < start[k + 1]; ++i) {
        const int s = lev[i];
        acc += (1.0 - ph[i]) * (xa[s] * xb[s]);
    }
    if (k > 0)
        for (int i = start[k - 1]; i < start[k]; ++i) {
            const int s = lev[i];
            acc += ph[i] * (xa[s] * xb[s]);
        }
    rho[(int64_t)k * nn + e] = acc;
}

// Forward transform rows: F[2q][k] = cos(2 pi k q / L), F[2q+1][k] = sin(...),
// q < Q, k < K.  The phase k q mod L is reduced exactly in integers.
__global__ void k_dft_fwd(int L, int Q, int K, double *__restrict__ F) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)2 * Q * K) return;
    const int r = (int)(idx / K), k = (int)(idx % K), q = r >> 1;
    const int64_t ph = ((int64_t)k * q) % L;
    double sn, cs;
    sincospi(2.0 * (double)ph / (double)L, &sn, &cs);
    F[idx] = (r & 1) ? sn : cs;
}

// Inverse transform of a real sequence from its first Q = L/2 + 1 transform
// values: a[m] = (1/L) sum_q c_q (Re A_q cos(2 pi m q / L) + Im A_q sin(...)),
// c_0 = c_{L/2} = 1, else 2.  G[m][2q] and G[m][2q+1] hold the two factors.
__global__ void k_dft_inv(int L, int Q, int M, double *__restrict__ G) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * 2 * Q) return;
    const int m = (int)(idx / (2 * Q)), c = (int)(idx % (2 * Q)), q = c >> 1;
    const int64_t ph = ((int64_t)m * q) % L;
    double sn, cs;
    sincospi(2.0 * (double)ph / (double)L, &sn, &cs);
    const double w = ((q == 0 || 2 * q == L) ? 1.0 : 2.0) / (double)L;
    G[idx] = w * ((c & 1) ? sn : cs);
}

constexpr int TO = TIME_MAX_ORB;
constexpr int TP = TO + 1;            // LDS row pitch (doubles)
constexpr int TC_NT = 512;            // threads per workgroup
constexpr int TC_FIXED = 8 * TO * TP;  // doubles of the fixed LDS part

// One workgroup per (block pair B1 <= B2, time point q0 + blockIdx.y).
// rho^+_{O1 O2}(t) and rhobar^-_{O2 O1}(t) are gathered into LDS, and the
// vertex matrices of the products of B1 are staged in LDS (mc at a time); for
// every product nu of B2: Y = rho^+ V_nu, M = Y rhobar^- (|O1| x |O1|), then
// a_{mu nu}(t) = 2 sum_{ab} V_mu^{ab} M_{ba} for the staged mu (mu <= nu), one
// wave per mu.  Output: Ahat[2 qq][t] = Re, Ahat[2 qq + 1][t] = Im, qq the
// time index within the chunk, t the packed upper index of (mu, nu).
// Dynamic LDS: TC_FIXED + mc |O1|^2 doubles.
__global__ __launch_bounds__(TC_NT) void k_time_contract(
    int n_orb, int n_prod, int q0, int v_cap, const int32_t *__restrict__ blk_prod,
    const int32_t *__restrict__ blk_orb, const int32_t *__restrict__ orb_idx, const int64_t *__restrict__ blk_val,
    const double *__restrict__ vals, const int32_t *__restrict__ pb1, const int32_t *__restrict__ pb2,
    const double *__restrict__ Rp, const double *__restrict__ Rm, double *__restrict__ Ahat, int64_t n_upper) {
    extern __shared__ double sm[];
    __shared__ int o1[TO], o2[TO];
    double *pr = sm, *pim = pr + TO * TP;    // rho^+_{O1 O2}: [i][j]
    double *mr = pim + TO * TP, *mim = mr + TO * TP;  // rhobar^-_{O2 O1}: [j][i]
    double *zr = mim + TO * TP, *zim = zr + TO * TP;  // V_nu [c][d] (zr), then M [b][a]
    double *yr = zim + TO * TP, *yim = yr + TO * TP;  // Y [i][d]
    double *v1s = sm + TC_FIXED;                       // V_mu of the staged products of B1
    const int B1 = pb1[blockIdx.x], B2 = pb2[blockIdx.x];
    const int qq = blockIdx.y, q = q0 + qq;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = TC_NT / 64;
    const int ob1 = blk_orb[B1], ob2 = blk_orb[B2];
    const int n1 = blk_orb[B1 + 1] - ob1, n2 = blk_orb[B2 + 1] - ob2;
    if (tid < n1) o1[tid] = orb_idx[ob1 + tid];
    if (tid < n2) o2[tid] = orb_idx[ob2 + tid];
    __syncthreads();
    const int64_t nn = (int64_t)n_orb * n_orb;
    const double *rpr = Rp + (int64_t)(2 * q) * nn, *rpi = rpr + nn;
    const double *rmr = Rm + (int64_t)(2 * q) * nn, *rmi = rmr + nn;
    for (int idx = tid; idx < n1 * n2; idx += TC_NT) {
        const int i = idx / n2, j = idx % n2;
        const int64_t ac = (int64_t)o1[i] * n_orb + o2[j], ca = (int64_t)o2[j] * n_orb + o1[i];
        pr[i * TP + j] = rpr[ac];
        pim[i * TP + j] = rpi[ac];
        mr[j * TP + i] = rmr[ca];
        mim[j * TP + i] = rmi[ca];
    }
    const int p1 = blk_prod[B1], e1 = blk_prod[B1 + 1];
    const int p2 = blk_prod[B2], e2 = blk_prod[B2 + 1];
    const int nsq1 = n1 * n1, nsq2 = n2 * n2;
    const int mc = max(1, v_cap / nsq1);
    const double *v1 = vals + blk_val[B1];
    const double *v2 = vals + blk_val[B2];
    double *ar = Ahat + (int64_t)(2 * qq) * n_upper, *ai = ar + n_upper;
    for (int c0 = p1; c0 < e1; c0 += mc) {
        const int c1 = min(e1, c0 + mc);
        __syncthreads();
        for (int idx = tid; idx < (c1 - c0) * nsq1; idx += TC_NT) v1s[idx] = v1[(int64_t)(c0 - p1) * nsq1 + idx];
        // with B1 == B2 only nu >= mu is needed
        for (int nu = (B1 == B2) ? c0 : p2; nu < e2; ++nu) {
            __syncthreads();
            const double *vnu = v2 + (int64_t)(nu - p2) * nsq2;
            for (int idx = tid; idx < nsq2; idx += TC_NT) zr[(idx / n2) * TP + idx % n2] = vnu[idx];
            __syncthreads();
            for (int idx = tid; idx < n1 * n2; idx += TC_NT) {
                const int i = idx / n2, d = idx % n2;
                double sr = 0.0, si = 0.0;
                for (int c = 0; c < n2; ++c) {
                    const double v = zr[c * TP + d];
                    sr += pr[i * TP + c] * v;
                    si += pim[i * TP + c] * v;
                }
                yr[i * TP + d] = sr;
                yim[i * TP + d] = si;
            }
            __syncthreads();
            for (int idx = tid; idx < nsq1; idx += TC_NT) {
                const int b = idx / n1, a = idx % n1;
                double sr = 0.0, si = 0.0;
                for (int d = 0; d < n2; ++d) {
                    const double xr = yr[b * TP + d], xi = yim[b * TP + d], wr = mr[d * TP + a], wi = mim[d * TP + a];
                    sr += xr * wr - xi * wi;
                    si += xr * wi + xi * wr;
                }
                zr[b * TP + a] = sr;
                zim[b * TP + a] = si;
            }
            __syncthreads();
            const int mu_end = (B1 == B2) ? min(c1, nu + 1) : c1;
            for (int mu = c0 + wave; mu < mu_end; mu += NW) {
                const double *vmu = v1s + (mu - c0) * nsq1;
                double sr = 0.0, si = 0.0;
                for (int e = lane; e < nsq1; e += 64) {
                    const int a = e / n1, b = e % n1;
                    const double v = vmu[e];
                    sr += v * zr[b * TP + a];
                    si += v * zim[b * TP + a];
                }
                for (int off = 32; off > 0; off >>= 1) {
                    sr += __shfl_xor(sr, off);
                    si += __shfl_xor(si, off);
                }
                if (lane == 0) {
                    const int64_t t = (int64_t)mu * n_prod - ((int64_t)mu * (mu - 1)) / 2 + (nu - mu);
                    ar[t] = 2.0 * sr;
                    ai[t] = 2.0 * si;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_rho_bins(hipStream_t st, int n_orb, int K, const double *X, const int32_t *lev, const double *ph,
                           const int32_t *start, double *rho) {
    const int64_t nn = (int64_t)n_orb * n_orb;
    if (K <= 0) return hipSuccess;
    ProfScope ps(st, "rho_bins", 0.0, 8.0 * K * (double)nn);
    hipLaunchKernelGGL(k_rho_bins, dim3((unsigned)((nn + 255) / 256), (unsigned)K), dim3(256), 0, st, n_orb, X, lev,
                       ph, start, rho);
    return hipGetLastError();
}

hipError_t launch_dft_matrices(hipStream_t st, int L, int Q, int K, double *F, int M, double *G) {
    if (F && K > 0) {
        const int64_t tot = (int64_t)2 * Q * K;
        hipLaunchKernelGGL(k_dft_fwd, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, Q, K, F);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (G && M > 0) {
        const int64_t tot = (int64_t)M * 2 * Q;
        hipLaunchKernelGGL(k_dft_inv, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, Q, M, G);
    }
    return hipGetLastError();
}

hipError_t launch_time_contract(hipStream_t st, int n_orb, int n_prod, int n_pairs_blk, int q0, int nq,
                                const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                const double *Rp, const double *Rm, double *Ahat, int max_vblock, double flops) {
    if (n_pairs_blk <= 0 || nq <= 0) return hipSuccess;
    const int64_t n_upper = (int64_t)n_prod * (n_prod + 1) / 2;
    // vertex staging: every product of the largest block if it fits in
    // 158 KB of LDS with the fixed part, else as many as fit
    const int cap_lds = 158 * 1024 / 8 - TC_FIXED;
    const int v_cap = std::max(TO * TO, std::min(max_vblock, cap_lds));
    const size_t lds = sizeof(double) * (size_t)(TC_FIXED + v_cap);
    hipError_t e = hipFuncSetAttribute((const void *)k_time_contract, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    ProfScope ps(st, "time_contract", flops, 16.0 * nq * (double)n_upper);
    hipLaunchKernelGGL(k_time_contract, dim3((unsigned)n_pairs_blk, (unsigned)nq), dim3(TC_NT), lds, st, n_orb, n_prod,
                       q0, v_cap, blk_prod, blk_orb, orb_idx, blk_val, vals, pb1, pb2, Rp, Rm, Ahat, n_upper);
    return hipGetLastError();
}

}  // namespace gwk
