// The GW self-energy downstream of W (Section 5.A eqs. spectral_3 and
// Cauchy1, evaluated time by time as in Section 8.B; Section 4 eq.
// instantaneous).  gamma, the spectral weight of W - v on the mesh, and the
// electronic densities rho+ and rhobar- are transformed to time; per time
// and per pair of vertex blocks the product
//   sigma^{ab}(t) += sum_{mu in B1, nu in B2} gamma^{mu nu}(t) (V_mu rho(t) V_nu)^{ab}
// is accumulated, and the sum is transformed back to the mesh.
#include "gw_internal.h"
#include "gw_prof.h"

#include <algorithm>

namespace gwk {
namespace {

// gamma[k][t] = -(d / pi) Im W[j0 + k][mu][nu] for the packed upper index t of
// (mu <= nu); gamma[0] = 0.  One workgroup per (row mu, bin k).
__global__ __launch_bounds__(256) void k_w_spectral(int n, int j0, double scale, const zdbl *__restrict__ W,
                                                    double *__restrict__ gam) {
    const int mu = blockIdx.x, k = blockIdx.y;
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    const int64_t row = (int64_t)mu * n - ((int64_t)mu * (mu - 1)) / 2 - mu;
    const zdbl *w = W + (int64_t)(j0 + k) * n * n + (int64_t)mu * n;
    double *g = gam + (int64_t)k * n_upper + row;
    for (int nu = mu + threadIdx.x; nu < n; nu += 256) g[nu] = (k == 0) ? 0.0 : scale * w[nu].im;
}

// dst[t] = src[mu][nu] for the packed upper index t of (mu <= nu).
__global__ __launch_bounds__(256) void k_pack_upper(int n, const double *__restrict__ src, double *__restrict__ dst) {
    const int mu = blockIdx.x;
    const int64_t row = (int64_t)mu * n - ((int64_t)mu * (mu - 1)) / 2 - mu;
    for (int nu = mu + threadIdx.x; nu < n; nu += 256) dst[row + nu] = src[(int64_t)mu * n + nu];
}

// Kp[j][m] = 1 / (w_j - m d + i eps), Km[j][m] = 1 / (w_j + m d + i eps), w_j = w0 + j d.
__global__ void k_cauchy_pm(int n_om, int M, double w0, double d, double eps, zdbl *__restrict__ Kp,
                            zdbl *__restrict__ Km) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_om * M) return;
    const int j = (int)(idx / M), m = (int)(idx % M);
    const double w = w0 + j * d, s = m * d, e2 = eps * eps;
    const double a = w - s, b = w + s;
    const double da = a * a + e2, db = b * b + e2;
    Kp[idx] = zdbl{a / da, -eps / da};
    Km[idx] = zdbl{b / db, -eps / db};
}

__global__ void k_scale_copy(int64_t n, double alpha, const double *__restrict__ src, double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = alpha * src[i];
}

constexpr int SO = TIME_MAX_ORB;
constexpr int SP = SO + 1;
constexpr int SC_NT = 512;

// One workgroup per (block pair B1 <= B2, time point q0 + blockIdx.y).  For
// every product mu of B1: G = sum_{nu in B2} gammahat^{mu nu} V_nu (|O2| x |O2|),
// U+- = rho+-_{O1 O2} G, C+- += V_mu U+-.  C+- is then added (atomically:
// several block pairs share orbitals) to S+-[qq][O1][O2] and, for B1 < B2,
// its transpose to S+-[qq][O2][O1] (the ordered pair (B2, B1)).  TWO = false:
// one density only (Rm, Sm unused).  Rp, Rm: [2Q][n_orb^2] (Re, Im planes per
// time point); Gh: [2 nq][n_upper]; S+-: [2 nq][n_orb^2].
template <bool TWO>
__global__ __launch_bounds__(SC_NT) void k_sigma_contract(
    int n_orb, int n_prod, int q0, const int32_t *__restrict__ blk_prod, const int32_t *__restrict__ blk_orb,
    const int32_t *__restrict__ orb_idx, const int64_t *__restrict__ blk_val, const double *__restrict__ vals,
    const int32_t *__restrict__ pb1, const int32_t *__restrict__ pb2, const double *__restrict__ Rp,
    const double *__restrict__ Rm, const double *__restrict__ Gh, double *__restrict__ Sp, double *__restrict__ Sm) {
    __shared__ int o1[SO], o2[SO];
    __shared__ double ppr[SO * SP], ppi[SO * SP], pmr[SO * SP], pmi[SO * SP];  // rho+- [a'][c], a' in O1, c in O2
    __shared__ double gr[SO * SP], gi[SO * SP];                                // G [c][d], O2 x O2
    __shared__ double upr[SO * SP], upi[SO * SP], umr[SO * SP], umi[SO * SP];  // U+- [a'][d]
    __shared__ double vm[SO * SP];                                             // V_mu [a][a']
    const int B1 = pb1[blockIdx.x], B2 = pb2[blockIdx.x];
    const int qq = blockIdx.y, q = q0 + qq;
    const int tid = threadIdx.x;
    const int ob1 = blk_orb[B1], ob2 = blk_orb[B2];
    const int n1 = blk_orb[B1 + 1] - ob1, n2 = blk_orb[B2 + 1] - ob2;
    if (tid < n1) o1[tid] = orb_idx[ob1 + tid];
    if (tid < n2) o2[tid] = orb_idx[ob2 + tid];
    __syncthreads();
    const int64_t nn = (int64_t)n_orb * n_orb;
    const int64_t n_upper = (int64_t)n_prod * (n_prod + 1) / 2;
    {
        const double *ar = Rp + (int64_t)(2 * q) * nn, *ai = ar + nn;
        const double *br = TWO ? Rm + (int64_t)(2 * q) * nn : nullptr, *bi = TWO ? br + nn : nullptr;
        for (int idx = tid; idx < n1 * n2; idx += SC_NT) {
            const int i = idx / n2, j = idx % n2;
            const int64_t ac = (int64_t)o1[i] * n_orb + o2[j];
            ppr[i * SP + j] = ar[ac];
            ppi[i * SP + j] = ai[ac];
            if (TWO) {
                pmr[i * SP + j] = br[ac];
                pmi[i * SP + j] = bi[ac];
            }
        }
    }
    const int p1 = blk_prod[B1], e1 = blk_prod[B1 + 1];
    const int p2 = blk_prod[B2], e2 = blk_prod[B2 + 1];
    const int nsq1 = n1 * n1, nsq2 = n2 * n2, n12 = n1 * n2;
    const double *v1 = vals + blk_val[B1];
    const double *v2 = vals + blk_val[B2];
    const double *ghr = Gh + (int64_t)(2 * qq) * n_upper, *ghi = ghr + n_upper;
    // this thread's elements (a, b) of C: e = tid + SC_NT r, r < 2 (n1 n2 <= 1024)
    double cpr[2] = {0.0, 0.0}, cpi[2] = {0.0, 0.0}, cmr[2] = {0.0, 0.0}, cmi[2] = {0.0, 0.0};
    for (int mu = p1; mu < e1; ++mu) {
        __syncthreads();
        const double *vmu = v1 + (int64_t)(mu - p1) * nsq1;
        for (int idx = tid; idx < nsq1; idx += SC_NT) vm[(idx / n1) * SP + idx % n1] = vmu[idx];
        // G = sum_nu gammahat^{mu nu} V_nu
        for (int idx = tid; idx < nsq2; idx += SC_NT) {
            double sr = 0.0, si = 0.0;
            for (int nu = p2; nu < e2; ++nu) {
                const int a = min(mu, nu), b = max(mu, nu);
                const int64_t t = (int64_t)a * n_prod - ((int64_t)a * (a - 1)) / 2 + (b - a);
                const double v = v2[(int64_t)(nu - p2) * nsq2 + idx];
                sr += ghr[t] * v;
                si += ghi[t] * v;
            }
            gr[(idx / n2) * SP + idx % n2] = sr;
            gi[(idx / n2) * SP + idx % n2] = si;
        }
        __syncthreads();
        // U+- = rho+- G
        for (int idx = tid; idx < n12; idx += SC_NT) {
            const int i = idx / n2, d = idx % n2;
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            for (int c = 0; c < n2; ++c) {
                const double xr = gr[c * SP + d], xi = gi[c * SP + d];
                const double pr = ppr[i * SP + c], pi = ppi[i * SP + c];
                ar += pr * xr - pi * xi;
                ai += pr * xi + pi * xr;
                if (TWO) {
                    const double mr = pmr[i * SP + c], mi = pmi[i * SP + c];
                    br += mr * xr - mi * xi;
                    bi += mr * xi + mi * xr;
                }
            }
            upr[i * SP + d] = ar;
            upi[i * SP + d] = ai;
            if (TWO) {
                umr[i * SP + d] = br;
                umi[i * SP + d] = bi;
            }
        }
        __syncthreads();
        // C+- += V_mu U+-
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = tid + SC_NT * r;
            if (e < n12) {
                const int a = e / n2, b = e % n2;
                double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                for (int k = 0; k < n1; ++k) {
                    const double v = vm[a * SP + k];
                    ar += v * upr[k * SP + b];
                    ai += v * upi[k * SP + b];
                    if (TWO) {
                        br += v * umr[k * SP + b];
                        bi += v * umi[k * SP + b];
                    }
                }
                cpr[r] += ar;
                cpi[r] += ai;
                if (TWO) {
                    cmr[r] += br;
                    cmi[r] += bi;
                }
            }
        }
    }
    double *spr = Sp + (int64_t)(2 * qq) * nn, *spi = spr + nn;
    double *smr = TWO ? Sm + (int64_t)(2 * qq) * nn : nullptr, *smi = TWO ? smr + nn : nullptr;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int e = tid + SC_NT * r;
        if (e < n12) {
            const int a = o1[e / n2], b = o2[e % n2];
            const int64_t ab = (int64_t)a * n_orb + b, ba = (int64_t)b * n_orb + a;
            atomicAdd(spr + ab, cpr[r]);
            atomicAdd(spi + ab, cpi[r]);
            if (TWO) {
                atomicAdd(smr + ab, cmr[r]);
                atomicAdd(smi + ab, cmi[r]);
            }
            if (B1 != B2) {
                atomicAdd(spr + ba, cpr[r]);
                atomicAdd(spi + ba, cpi[r]);
                if (TWO) {
                    atomicAdd(smr + ba, cmr[r]);
                    atomicAdd(smi + ba, cmi[r]);
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_w_spectral(hipStream_t st, int n, int n_sb, int j0, double domega, const zdbl *W, double *gam) {
    if (n_sb <= 0) return hipSuccess;
    const double scale = -domega / 3.14159265358979323846;
    hipLaunchKernelGGL(k_w_spectral, dim3((unsigned)n, (unsigned)n_sb), dim3(256), 0, st, n, j0, scale, W, gam);
    return hipGetLastError();
}

hipError_t launch_pack_upper(hipStream_t st, int n, const double *src, double *dst) {
    hipLaunchKernelGGL(k_pack_upper, dim3((unsigned)n), dim3(256), 0, st, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_cauchy_pm(hipStream_t st, int n_om, int M, double w0, double d, double eps, zdbl *Kp, zdbl *Km) {
    const int64_t tot = (int64_t)n_om * M;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cauchy_pm, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_om, M, w0, d, eps, Kp,
                       Km);
    return hipGetLastError();
}

hipError_t launch_scale_copy(hipStream_t st, int64_t n, double alpha, const double *src, double *dst) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)blocks), dim3(256), 0, st, n, alpha, src, dst);
    return hipGetLastError();
}

hipError_t launch_sigma_contract(hipStream_t st, int n_orb, int n_prod, int n_pairs_blk, int q0, int nq,
                                 const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                 const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                 const double *Rp, const double *Rm, const double *Gh, double *Sp, double *Sm,
                                 double flops) {
    if (n_pairs_blk <= 0 || nq <= 0) return hipSuccess;
    const double nn = (double)n_orb * n_orb;
    ProfScope ps(st, "sigma_contract", flops, 16.0 * nq * nn * (Rm ? 2 : 1));
    dim3 grid((unsigned)n_pairs_blk, (unsigned)nq);
    if (Rm)
        hipLaunchKernelGGL(k_sigma_contract<true>, grid, dim3(SC_NT), 0, st, n_orb, n_prod, q0, blk_prod, blk_orb,
                           orb_idx, blk_val, vals, pb1, pb2, Rp, Rm, Gh, Sp, Sm);
    else
        hipLaunchKernelGGL(k_sigma_contract<false>, grid, dim3(SC_NT), 0, st, n_orb, n_prod, q0, blk_prod, blk_orb,
                           orb_idx, blk_val, vals, pb1, pb2, Rp, (const double *)nullptr, Gh, Sp, (double *)nullptr);
    return hipGetLastError();
}

}  // namespace gwk
