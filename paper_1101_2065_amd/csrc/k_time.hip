// The paper's own route to the spectral function of the free response
// (Section 8.A eq. sf-of-response-time): the electronic densities of Section 5
// split into empty (rho^+) and occupied (rhobar^-(s) = rho^-(-s)) parts on the
// mesh, their Fourier transforms to time, the local product
//   a_{mu nu}(t) = 2 V_mu^{ab} rho^+_{bc}(t) V_nu^{cd} rhobar^-_{da}(t)
// time by time (small products on the matrix cores), and the transform back
// to the mesh.  On the mesh the two
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
constexpr int TP = TO + 1;  // LDS row pitch (doubles)

typedef double v4d __attribute__((ext_vector_type(4)));
__device__ inline v4d mfma4(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// One wave's share of a (block pair, time point): for each of its products nu
// of B2 (nu = p2 + wave, step 4)
//   Y^T = V_nu (rho+)^T  (|O2| x |O1|), M = Y rhobar-  (|O1| x |O1|),
//   a_{mu nu} = 2 sum_{i,a} V_mu^{ai} M_{ia} for every mu of B1 (mu <= nu),
// all on the matrix cores in 16 x 16 tiles (T1, T2 tiles for O1, O2, zero
// padded).  f64 16x16x4 layouts (gfx950): A operand lane l = A[l % 16][l / 16],
// B operand lane l = B[l / 16][l % 16], result element e of lane l =
// D[l / 16 + 4 e][l % 16].  The result of Y^T = V P^T is therefore already the
// A operand of Y R (element e = k step e of each 16-wide block of d), so Y never
// leaves the registers.
template <int T1, int T2>
__device__ void time_wave(int n1, int n2, int p1, int e1, int p2, int e2, bool same, int n_prod, int lane, int wave,
                          const double *__restrict__ v1, const double *__restrict__ v2, const double *pr,
                          const double *pim, const double *mr_, const double *mim, double *__restrict__ ar,
                          double *__restrict__ ai) {
    const int lr = lane & 15, lk = lane >> 4;
    const int nsq1 = n1 * n1, nsq2 = n2 * n2;
    for (int nu = p2 + wave; nu < e2; nu += 4) {
        const double *vnu = v2 + (int64_t)(nu - p2) * nsq2;
        // Y^T[d][i] = sum_c V[d][c] P[i][c]; the V_nu operands of every k step
        // are loaded up front so one memory latency covers them all
        double va[4 * T2][T2];
#pragma unroll
        for (int s = 0; s < 4 * T2; ++s)
#pragma unroll
            for (int dt = 0; dt < T2; ++dt) {
                const int c = 4 * s + lk, d = dt * 16 + lr;
                va[s][dt] = (d < n2 && c < n2) ? vnu[d * n2 + c] : 0.0;
            }
        v4d ytr[T2][T1], yti[T2][T1];
#pragma unroll
        for (int dt = 0; dt < T2; ++dt)
#pragma unroll
            for (int it = 0; it < T1; ++it) ytr[dt][it] = yti[dt][it] = v4d{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4 * T2; ++s) {
            const int c = 4 * s + lk;
            double pbr[T1], pbi[T1];
#pragma unroll
            for (int it = 0; it < T1; ++it) {
                const int i = it * 16 + lr;
                pbr[it] = pr[i * TP + c];
                pbi[it] = pim[i * TP + c];
            }
#pragma unroll
            for (int dt = 0; dt < T2; ++dt)
#pragma unroll
                for (int it = 0; it < T1; ++it) {
                    ytr[dt][it] = mfma4(va[s][dt], pbr[it], ytr[dt][it]);
                    yti[dt][it] = mfma4(va[s][dt], pbi[it], yti[dt][it]);
                }
        }
        // M[i][a] = sum_d Y[i][d] R[d][a]
        v4d mr[T1][T1], mi[T1][T1];
#pragma unroll
        for (int it = 0; it < T1; ++it)
#pragma unroll
            for (int at = 0; at < T1; ++at) mr[it][at] = mi[it][at] = v4d{0, 0, 0, 0};
#pragma unroll
        for (int dt = 0; dt < T2; ++dt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int d = dt * 16 + 4 * e + lk;
                double rbr[T1], rbi[T1];
#pragma unroll
                for (int at = 0; at < T1; ++at) {
                    rbr[at] = mr_[d * TP + at * 16 + lr];
                    rbi[at] = mim[d * TP + at * 16 + lr];
                }
#pragma unroll
                for (int it = 0; it < T1; ++it) {
                    const double yr = ytr[dt][it][e], yi = yti[dt][it][e];
#pragma unroll
                    for (int at = 0; at < T1; ++at) {
                        mr[it][at] = mfma4(yr, rbr[at], mr[it][at]);
                        mr[it][at] = mfma4(-yi, rbi[at], mr[it][at]);
                        mi[it][at] = mfma4(yr, rbi[at], mi[it][at]);
                        mi[it][at] = mfma4(yi, rbr[at], mi[it][at]);
                    }
                }
            }
        // traces with the vertex matrices of B1, 16 products mu at a time: lane
        // holds M[i][a] at i = it*16 + lk + 4e, a = at*16 + lr; its partial sums
        // for the 16 mu (re, im: 32 values) are reduced over the wave by a
        // butterfly that halves the values per lane at every step, so the 16
        // totals take 31 exchanges and 6 dependent steps instead of 16 x 12
        const int mu_end = same ? nu + 1 : e1;
        for (int m0 = p1; m0 < mu_end; m0 += 16) {
            double v[32];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int mu = m0 + m;
                double sr = 0.0, si = 0.0;
                if (mu < mu_end) {
                    const double *vmu = v1 + (int64_t)(mu - p1) * nsq1;
#pragma unroll
                    for (int it = 0; it < T1; ++it)
#pragma unroll
                        for (int at = 0; at < T1; ++at)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int ii = it * 16 + lk + 4 * e, a = at * 16 + lr;
                                const double x = (ii < n1 && a < n1) ? vmu[ii * n1 + a] : 0.0;
                                sr += x * mr[it][at][e];
                                si += x * mi[it][at][e];
                            }
                }
                v[2 * m] = sr;
                v[2 * m + 1] = si;
            }
#pragma unroll
            for (int step = 0, half = 16; step < 5; ++step, half >>= 1) {
                const int bit = 32 >> step;  // lane bit deciding which half this lane keeps
                const bool up = (lane & bit) != 0;
#pragma unroll
                for (int j = 0; j < half; ++j) {
                    const double send = up ? v[j] : v[j + half];
                    const double keep = up ? v[j + half] : v[j];
                    v[j] = keep + __shfl_xor(send, bit);
                }
            }
            v[0] += __shfl_xor(v[0], 1);
            // lane l now holds value (l >> 1) & 31: product m0 + ((l >> 2) & 15), part (l >> 1) & 1
            const int idx = (lane >> 1) & 31, mu = m0 + (idx >> 1);
            if ((lane & 1) == 0 && mu < mu_end) {
                const int64_t t = (int64_t)mu * n_prod - ((int64_t)mu * (mu - 1)) / 2 + (nu - mu);
                (idx & 1 ? ai : ar)[t] = 2.0 * v[0];
            }
        }
    }
}

// One workgroup (4 waves) per (time point q0 + blockIdx.x, block pair
// B1 <= B2 of blockIdx.y): rho+_{O1 O2}(t) and rhobar-_{O2 O1}(t) are gathered into LDS
// (zero padded to whole 16-tiles), then every wave works through its own
// products nu with no further barrier.  Output: Ahat[2 qq][t] = Re,
// Ahat[2 qq + 1][t] = Im, qq the time index within the chunk, t the packed
// upper index of (mu, nu).
template <int T1, int T2>
__global__ __launch_bounds__(256) void k_time_contract(
    int n_orb, int n_prod, int q0, const int32_t *__restrict__ blk_prod, const int32_t *__restrict__ blk_orb,
    const int32_t *__restrict__ orb_idx, const int64_t *__restrict__ blk_val, const double *__restrict__ vals,
    const int32_t *__restrict__ pb1, const int32_t *__restrict__ pb2, const double *__restrict__ Rp,
    const double *__restrict__ Rm, double *__restrict__ Ahat, int64_t n_upper) {
    __shared__ int o1[TO], o2[TO];
    __shared__ double pr[TO * TP], pim[TO * TP];  // rho+ [i][c], i in O1, c in O2
    __shared__ double mr[TO * TP], mim[TO * TP];  // rhobar- [d][a], d in O2, a in O1
    // time points fastest, so that neighbouring workgroups share the vertex
    // blocks in the L2
    const int B1 = pb1[blockIdx.y], B2 = pb2[blockIdx.y];
    const int qq = blockIdx.x, q = q0 + qq;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ob1 = blk_orb[B1], ob2 = blk_orb[B2];
    const int n1 = blk_orb[B1 + 1] - ob1, n2 = blk_orb[B2 + 1] - ob2;
    if (tid < n1) o1[tid] = orb_idx[ob1 + tid];
    if (tid < n2) o2[tid] = orb_idx[ob2 + tid];
    for (int idx = tid; idx < TO * TP; idx += 256) pr[idx] = pim[idx] = mr[idx] = mim[idx] = 0.0;
    __syncthreads();
    const int64_t nn = (int64_t)n_orb * n_orb;
    const double *rpr = Rp + (int64_t)(2 * q) * nn, *rpi = rpr + nn;
    const double *rmr = Rm + (int64_t)(2 * q) * nn, *rmi = rmr + nn;
    for (int idx = tid; idx < n1 * n2; idx += 256) {
        const int i = idx / n2, j = idx % n2;
        const int64_t ac = (int64_t)o1[i] * n_orb + o2[j], ca = (int64_t)o2[j] * n_orb + o1[i];
        pr[i * TP + j] = rpr[ac];
        pim[i * TP + j] = rpi[ac];
        mr[j * TP + i] = rmr[ca];
        mim[j * TP + i] = rmi[ca];
    }
    __syncthreads();
    const int p1 = blk_prod[B1], e1 = blk_prod[B1 + 1];
    const int p2 = blk_prod[B2], e2 = blk_prod[B2 + 1];
    const double *v1 = vals + blk_val[B1];
    const double *v2 = vals + blk_val[B2];
    double *ar = Ahat + (int64_t)(2 * qq) * n_upper, *ai = ar + n_upper;
    time_wave<T1, T2>(n1, n2, p1, e1, p2, e2, B1 == B2, n_prod, lane, wave, v1, v2, pr, pim, mr, mim, ar, ai);
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

hipError_t launch_time_contract(hipStream_t st, int n_orb, int n_prod, const int *class_off, int q0, int nq,
                                const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                const double *Rp, const double *Rm, double *Ahat, double flops) {
    if (class_off[4] <= 0 || nq <= 0) return hipSuccess;
    const int64_t n_upper = (int64_t)n_prod * (n_prod + 1) / 2;
    ProfScope ps(st, "time_contract", flops, 16.0 * nq * (double)n_upper);
    // one launch per tile class (|O1|, |O2| up to 16 or 32): each instance
    // keeps only the registers its tiles need
#define GW_TC(T1, T2, c)                                                                                          \
    if (class_off[c + 1] > class_off[c])                                                                         \
        hipLaunchKernelGGL((k_time_contract<T1, T2>), dim3((unsigned)nq, (unsigned)(class_off[c + 1] - class_off[c])), \
                           dim3(256), 0, st, n_orb, n_prod, q0, blk_prod, blk_orb, orb_idx, blk_val, vals,        \
                           pb1 + class_off[c], pb2 + class_off[c], Rp, Rm, Ahat, n_upper);
    GW_TC(1, 1, 0)
    GW_TC(1, 2, 1)
    GW_TC(2, 1, 2)
    GW_TC(2, 2, 3)
#undef GW_TC
    return hipGetLastError();
}

}  // namespace gwk
