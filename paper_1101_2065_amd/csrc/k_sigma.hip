// The GW self-energy downstream of W (Section 5.A eqs. spectral_3 and
// Cauchy1, evaluated time by time as in Section 8.B; Section 4 eq.
// instantaneous).  gamma, the spectral weight of W - v on the mesh, and the
// electronic densities rho+ and rhobar- are transformed to time; per time
// and per pair of vertex blocks the product
//   sigma^{ab}(t) += sum_{mu in B1, nu in B2} gamma^{mu nu}(t) (V_mu rho(t) V_nu)^{ab}
// is accumulated (small products on the matrix cores), and the sum is
// transformed back to the mesh.
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

// Xe[a][E] = X[a][E] eig[E]
__global__ void k_scale_cols(int n, const double *__restrict__ X, const double *__restrict__ eig,
                             double *__restrict__ Xe) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    Xe[idx] = X[idx] * eig[idx % n];
}

// Hs = H + Sx - Vxc (either may be null)
__global__ void k_static_part(int64_t nn, const double *__restrict__ H, const double *__restrict__ Sx,
                              const double *__restrict__ Vxc, double *__restrict__ Hs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double h = H[i];
    if (Sx) h += Sx[i];
    if (Vxc) h -= Vxc[i];
    Hs[i] = h;
}

// A[b] = (w_{j0+b} + i eps) 1 - Hs - Sigma_c[j0+b]   (Sigma_c may be null)
__global__ void k_dyson_form(int n, int j0, double w0, double d, double eps, const double *__restrict__ Hs,
                             const zdbl *__restrict__ Sc, zdbl *__restrict__ A) {
    const int64_t nn = (int64_t)n * n;
    const int b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const int r = (int)(i / n), c = (int)(i % n);
    zdbl v{-Hs[i], 0.0};
    if (r == c) {
        v.re += w0 + (j0 + b) * d;
        v.im += eps;
    }
    if (Sc) {
        const zdbl s = Sc[(int64_t)(j0 + b) * nn + i];
        v.re -= s.re;
        v.im -= s.im;
    }
    A[(int64_t)b * nn + i] = v;
}

// dos[j0 + b] = -(1/pi) Im tr G[b]
__global__ __launch_bounds__(256) void k_trace_dos(int n, int j0, const zdbl *__restrict__ G, int64_t sG,
                                                   double *__restrict__ dos) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += G[(int64_t)b * sG + (int64_t)i * n + i].im;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) dos[j0 + b] = -red[0] / 3.14159265358979323846;
}

constexpr int SO = TIME_MAX_ORB;
constexpr int SP = SO + 1;

typedef double v4d __attribute__((ext_vector_type(4)));

// value of v in lane k (k wave-uniform)
__device__ inline double rlane_d(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k), hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline v4d mfma4(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// One wave's share of a (block pair, time point): for its products mu of B1
// (mu = p1 + wave, step 4)
//   G = sum_{nu in B2} gammahat^{mu nu} V_nu  (|O2| x |O2|, on the vector units,
//       computed directly in the B-operand layout),
//   U+- = rho+- G  (matrix cores), C+- += V_mu U+-  (matrix cores; U's result
//       layout is the B-operand layout of this product, and C accumulates in
//       the MFMA registers over mu).
// f64 16x16x4 layouts (gfx950): A operand lane l = A[l % 16][l / 16], B operand
// lane l = B[l / 16][l % 16], result element e of lane l = D[l / 16 + 4 e][l % 16].
// TWO = false: one density only.  The wave's C+- are then added to S+-
// (atomically; the transpose too for B1 < B2).
template <int T1, int T2, bool TWO>
__device__ void sigma_wave(int n1, int n2, int p1, int e1, int p2, int e2, bool same, int n_prod, int n_orb,
                           int lane, int wave, const double *__restrict__ v1, const double *v2,
                           const double *__restrict__ ghr, const double *__restrict__ ghi, const double *ppr,
                           const double *ppi, const double *pmr, const double *pmi, const int *o1, const int *o2,
                           double *spr, double *spi, double *smr, double *smi) {
    const int lr = lane & 15, lk = lane >> 4;
    const int nsq1 = n1 * n1, nsq2 = n2 * n2;
    v4d cpr[T1][T2], cpi[T1][T2], cmr[T1][T2], cmi[T1][T2];
#pragma unroll
    for (int at = 0; at < T1; ++at)
#pragma unroll
        for (int dt = 0; dt < T2; ++dt) cpr[at][dt] = cpi[at][dt] = cmr[at][dt] = cmi[at][dt] = v4d{0, 0, 0, 0};
    for (int mu = p1 + wave; mu < e1; mu += 4) {
        // G[c][d] at c = 4 s + lk, d = dt*16 + lr: the B operand of every k step
        double gr[4 * T2][T2], gi[4 * T2][T2];
#pragma unroll
        for (int s = 0; s < 4 * T2; ++s)
#pragma unroll
            for (int dt = 0; dt < T2; ++dt) gr[s][dt] = gi[s][dt] = 0.0;
        // the weights gammahat^{mu nu} of 64 products nu at a time, one per
        // lane (one vector load instead of a dependent load per nu)
        double lwr = 0.0, lwi = 0.0;
        for (int nu = p2; nu < e2; ++nu) {
            const int q = (nu - p2) & 63;
            if (q == 0) {
                const int nl = nu + lane;
                if (nl < e2) {
                    const int a = min(mu, nl), b = max(mu, nl);
                    const int64_t t = (int64_t)a * n_prod - ((int64_t)a * (a - 1)) / 2 + (b - a);
                    lwr = ghr[t];
                    lwi = ghi[t];
                }
            }
            const double wr = rlane_d(lwr, q), wi = rlane_d(lwi, q);
            const double *vnu = v2 + (int64_t)(nu - p2) * nsq2;  // LDS copy when staged
#pragma unroll
            for (int s = 0; s < 4 * T2; ++s)
#pragma unroll
                for (int dt = 0; dt < T2; ++dt) {
                    const int c = 4 * s + lk, d = dt * 16 + lr;
                    const double v = (c < n2 && d < n2) ? vnu[c * n2 + d] : 0.0;
                    gr[s][dt] += wr * v;
                    gi[s][dt] += wi * v;
                }
        }
        // vertex entries of mu, the A operand of C += V_mu U: V[a][i] at
        // a = at*16 + lr, i = 4 k + lk
        double va[T1][4 * T1];
        const double *vmu = v1 + (int64_t)(mu - p1) * nsq1;
#pragma unroll
        for (int at = 0; at < T1; ++at)
#pragma unroll
            for (int k = 0; k < 4 * T1; ++k) {
                const int a = at * 16 + lr, ii = 4 * k + lk;
                va[at][k] = (a < n1 && ii < n1) ? vmu[a * n1 + ii] : 0.0;
            }
#pragma unroll
        for (int den = 0; den < (TWO ? 2 : 1); ++den) {
            const double *qr = den ? pmr : ppr, *qi = den ? pmi : ppi;
            // U[i][d] = sum_c rho[i][c] G[c][d]
            v4d ur[T1][T2], ui[T1][T2];
#pragma unroll
            for (int it = 0; it < T1; ++it)
#pragma unroll
                for (int dt = 0; dt < T2; ++dt) ur[it][dt] = ui[it][dt] = v4d{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4 * T2; ++s) {
                const int c = 4 * s + lk;
#pragma unroll
                for (int it = 0; it < T1; ++it) {
                    const double ar = qr[(it * 16 + lr) * SP + c], ai = qi[(it * 16 + lr) * SP + c];
#pragma unroll
                    for (int dt = 0; dt < T2; ++dt) {
                        ur[it][dt] = mfma4(ar, gr[s][dt], ur[it][dt]);
                        ur[it][dt] = mfma4(-ai, gi[s][dt], ur[it][dt]);
                        ui[it][dt] = mfma4(ar, gi[s][dt], ui[it][dt]);
                        ui[it][dt] = mfma4(ai, gr[s][dt], ui[it][dt]);
                    }
                }
            }
            // C[a][d] += sum_i V[a][i] U[i][d]; k steps over i: tile it, element e
#pragma unroll
            for (int it = 0; it < T1; ++it)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int at = 0; at < T1; ++at)
#pragma unroll
                        for (int dt = 0; dt < T2; ++dt) {
                            const double a = va[at][4 * it + e];
                            if (den == 0) {
                                cpr[at][dt] = mfma4(a, ur[it][dt][e], cpr[at][dt]);
                                cpi[at][dt] = mfma4(a, ui[it][dt][e], cpi[at][dt]);
                            } else {
                                cmr[at][dt] = mfma4(a, ur[it][dt][e], cmr[at][dt]);
                                cmi[at][dt] = mfma4(a, ui[it][dt][e], cmi[at][dt]);
                            }
                        }
        }
    }
    // add this wave's C+- (element e of a lane: a = at*16 + lk + 4e, b = dt*16 + lr)
    const int64_t no = n_orb;
#pragma unroll
    for (int at = 0; at < T1; ++at)
#pragma unroll
        for (int dt = 0; dt < T2; ++dt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = at * 16 + lk + 4 * e, b = dt * 16 + lr;
                if (a < n1 && b < n2) {
                    const int64_t ab = (int64_t)o1[a] * no + o2[b], ba = (int64_t)o2[b] * no + o1[a];
                    atomicAdd(spr + ab, cpr[at][dt][e]);
                    atomicAdd(spi + ab, cpi[at][dt][e]);
                    if (TWO) {
                        atomicAdd(smr + ab, cmr[at][dt][e]);
                        atomicAdd(smi + ab, cmi[at][dt][e]);
                    }
                    if (!same) {
                        atomicAdd(spr + ba, cpr[at][dt][e]);
                        atomicAdd(spi + ba, cpi[at][dt][e]);
                        if (TWO) {
                            atomicAdd(smr + ba, cmr[at][dt][e]);
                            atomicAdd(smi + ba, cmi[at][dt][e]);
                        }
                    }
                }
            }
}

// One workgroup (4 waves) per (time point q0 + blockIdx.x, block pair
// B1 <= B2 of blockIdx.y); rho+- restricted to O1 x O2 are gathered into LDS
// (zero padded to whole 16-tiles).  Rp, Rm: [2Q][n_orb^2] (Re, Im planes per
// time point); Gh: [2 nq][n_upper]; S+-: [2 nq][n_orb^2].
template <int T1, int T2, bool TWO>
__global__ __launch_bounds__(256) void k_sigma_contract(
    int n_orb, int n_prod, int q0, int v_cap, const int32_t *__restrict__ blk_prod,
    const int32_t *__restrict__ blk_orb, const int32_t *__restrict__ orb_idx, const int64_t *__restrict__ blk_val,
    const double *__restrict__ vals, const int32_t *__restrict__ pb1, const int32_t *__restrict__ pb2,
    const double *__restrict__ Rp, const double *__restrict__ Rm, const double *__restrict__ Gh,
    double *__restrict__ Sp, double *__restrict__ Sm) {
    __shared__ int o1[SO], o2[SO];
    __shared__ double ppr[SO * SP], ppi[SO * SP], pmr[TWO ? SO * SP : 1], pmi[TWO ? SO * SP : 1];
    extern __shared__ double vstage[];  // V of B2, when it fits in v_cap doubles
    const int B1 = pb1[blockIdx.y], B2 = pb2[blockIdx.y];
    const int qq = blockIdx.x, q = q0 + qq;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ob1 = blk_orb[B1], ob2 = blk_orb[B2];
    const int n1 = blk_orb[B1 + 1] - ob1, n2 = blk_orb[B2 + 1] - ob2;
    if (tid < n1) o1[tid] = orb_idx[ob1 + tid];
    if (tid < n2) o2[tid] = orb_idx[ob2 + tid];
    for (int idx = tid; idx < SO * SP; idx += 256) {
        ppr[idx] = ppi[idx] = 0.0;
        if (TWO) pmr[idx] = pmi[idx] = 0.0;
    }
    __syncthreads();
    const int64_t nn = (int64_t)n_orb * n_orb;
    const int64_t n_upper = (int64_t)n_prod * (n_prod + 1) / 2;
    {
        const double *ar = Rp + (int64_t)(2 * q) * nn, *ai = ar + nn;
        const double *br = TWO ? Rm + (int64_t)(2 * q) * nn : nullptr, *bi = TWO ? br + nn : nullptr;
        for (int idx = tid; idx < n1 * n2; idx += 256) {
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
    const double *v2 = vals + blk_val[B2];
    const int nv2 = (blk_prod[B2 + 1] - blk_prod[B2]) * n2 * n2;
    if (nv2 <= v_cap) {
        for (int idx = tid; idx < nv2; idx += 256) vstage[idx] = v2[idx];
        v2 = vstage;
    }
    __syncthreads();
    const double *ghr = Gh + (int64_t)(2 * qq) * n_upper, *ghi = ghr + n_upper;
    double *spr = Sp + (int64_t)(2 * qq) * nn, *spi = spr + nn;
    double *smr = TWO ? Sm + (int64_t)(2 * qq) * nn : nullptr, *smi = TWO ? smr + nn : nullptr;
    sigma_wave<T1, T2, TWO>(n1, n2, blk_prod[B1], blk_prod[B1 + 1], blk_prod[B2], blk_prod[B2 + 1], B1 == B2, n_prod,
                            n_orb, lane, wave, vals + blk_val[B1], v2, ghr, ghi, ppr, ppi, pmr, pmi,
                            o1, o2, spr, spi, smr, smi);
}

}  // namespace

hipError_t launch_scale_cols(hipStream_t st, int n, const double *X, const double *eig, double *Xe) {
    const int64_t nn = (int64_t)n * n;
    hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, n, X, eig, Xe);
    return hipGetLastError();
}

hipError_t launch_static_part(hipStream_t st, int64_t nn, const double *H, const double *Sx, const double *Vxc,
                              double *Hs) {
    hipLaunchKernelGGL(k_static_part, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, nn, H, Sx, Vxc, Hs);
    return hipGetLastError();
}

hipError_t launch_dyson_form(hipStream_t st, int n, int j0, int nb, double w0, double d, double eps, const double *Hs,
                             const zdbl *Sc, zdbl *A) {
    const int64_t nn = (int64_t)n * n;
    ProfScope ps(st, "dyson_form", 0.0, 16.0 * 2.0 * nb * (double)nn);
    hipLaunchKernelGGL(k_dyson_form, dim3((unsigned)((nn + 255) / 256), (unsigned)nb), dim3(256), 0, st, n, j0, w0,
                       d, eps, Hs, Sc, A);
    return hipGetLastError();
}

hipError_t launch_trace_dos(hipStream_t st, int n, int j0, int nb, const zdbl *G, int64_t sG, double *dos) {
    hipLaunchKernelGGL(k_trace_dos, dim3((unsigned)nb), dim3(256), 0, st, n, j0, G, sG, dos);
    return hipGetLastError();
}

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

hipError_t launch_sigma_contract(hipStream_t st, int n_orb, int n_prod, const int *class_off, int q0, int nq,
                                 const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                 const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                 const double *Rp, const double *Rm, const double *Gh, double *Sp, double *Sm,
                                 int max_vblock, double flops) {
    if (class_off[4] <= 0 || nq <= 0) return hipSuccess;
    // the vertex block of B2 is staged in LDS when it fits next to the
    // densities (96 KB); larger blocks are read from memory
    const int v_cap = std::min(max_vblock, 96 * 1024 / 8);
    const size_t lds = sizeof(double) * (size_t)v_cap;
    const double nn = (double)n_orb * n_orb;
    ProfScope ps(st, "sigma_contract", flops, 16.0 * nq * nn * (Rm ? 2 : 1));
    // one launch per tile class (|O1|, |O2| up to 16 or 32)
#define GW_SC(T1, T2, c)                                                                                        \
    if (class_off[c + 1] > class_off[c]) {                                                                     \
        dim3 grid((unsigned)nq, (unsigned)(class_off[c + 1] - class_off[c]));                                  \
        hipError_t ea = Rm ? hipFuncSetAttribute((const void *)k_sigma_contract<T1, T2, true>,                  \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)           \
                           : hipFuncSetAttribute((const void *)k_sigma_contract<T1, T2, false>,                 \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);          \
        if (ea != hipSuccess) return ea;                                                                       \
        if (Rm)                                                                                                \
            hipLaunchKernelGGL((k_sigma_contract<T1, T2, true>), grid, dim3(256), lds, st, n_orb, n_prod, q0,    \
                               v_cap, blk_prod, blk_orb, orb_idx, blk_val, vals, pb1 + class_off[c],           \
                               pb2 + class_off[c], Rp, Rm, Gh, Sp, Sm);                                        \
        else                                                                                                   \
            hipLaunchKernelGGL((k_sigma_contract<T1, T2, false>), grid, dim3(256), lds, st, n_orb, n_prod, q0,   \
                               v_cap, blk_prod, blk_orb, orb_idx, blk_val, vals, pb1 + class_off[c],           \
                               pb2 + class_off[c], Rp, (const double *)nullptr, Gh, Sp, (double *)nullptr);    \
    }
    GW_SC(1, 1, 0)
    GW_SC(1, 2, 1)
    GW_SC(2, 1, 2)
    GW_SC(2, 2, 3)
#undef GW_SC
    return hipGetLastError();
}

}  // namespace gwk
