// chi0 from the histogram on gfx950: the Cauchy transform of the odd-extended
// spectral function as an FFT convolution with a precomputed kernel spectrum
// (Section 5.A eq. chi_by_spectra; Section 8.A does its convolutions by FFT).
#include "gw_internal.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace gwk {

namespace {

// ------------------------------------------------------------------ Cauchy kernel spectrum
// k(r) = 1/((r + j0) domega + i eps) for r in [0, 3L/4), and k(r - L) above
// (the negative lags); Kt = DFT_L(k) summed directly with exact argument
// reduction and compensated sums; tw[q] = exp(-2 pi i q / L).
__global__ void k_kspec(int L, int j0, double domega, double eps, zdbl *Kt, zdbl *tw) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= L) return;
    double sr = 0, si = 0, cr = 0, ci = 0;
    for (int r = 0; r < L; ++r) {
        const int lag = (r < (3 * L) / 4) ? r : r - L;
        const double x = (double)(lag + j0) * domega;
        const double den = x * x + eps * eps;
        const double kr = x / den, ki = -eps / den;
        const int64_t ph = ((int64_t)q * r) % L;
        double sn, cs;
        sincospi(2.0 * (double)ph / (double)L, &sn, &cs);
        // k * exp(-i theta) = (kr + i ki)(cs - i sn)
        const double tr = kr * cs + ki * sn;
        const double ti = ki * cs - kr * sn;
        double yr = tr - cr, t1 = sr + yr;
        cr = (t1 - sr) - yr;
        sr = t1;
        double yi = ti - ci, t2 = si + yi;
        ci = (t2 - si) - yi;
        si = t2;
    }
    Kt[q] = zdbl{sr, si};
    double sn, cs;
    sincospi(2.0 * (double)q / (double)L, &sn, &cs);
    tw[q] = zdbl{cs, -sn};
}

// ------------------------------------------------------------------ FFT (Stockham, LDS)
__device__ inline zdbl zmul(zdbl a, zdbl b) { return zdbl{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zdbl zadd(zdbl a, zdbl b) { return zdbl{a.re + b.re, a.im + b.im}; }
__device__ inline zdbl zsub(zdbl a, zdbl b) { return zdbl{a.re - b.re, a.im - b.im}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ inline zdbl rot90(zdbl a) { return INV ? zdbl{-a.im, a.re} : zdbl{a.im, -a.re}; }

template <bool INV>
__device__ inline void dft2(zdbl *v) {
    zdbl a = v[0], b = v[1];
    v[0] = zadd(a, b);
    v[1] = zsub(a, b);
}
template <bool INV>
__device__ inline void dft4(zdbl *v) {
    zdbl s02 = zadd(v[0], v[2]), d02 = zsub(v[0], v[2]);
    zdbl s13 = zadd(v[1], v[3]), d13 = rot90<INV>(zsub(v[1], v[3]));
    v[0] = zadd(s02, s13);
    v[2] = zsub(s02, s13);
    v[1] = zadd(d02, d13);
    v[3] = zsub(d02, d13);
}
template <bool INV>
__device__ inline void dft8(zdbl *v) {
    constexpr double h = 0.70710678118654752440;
    zdbl e[4] = {v[0], v[2], v[4], v[6]};
    zdbl o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // twiddles W8^k, k = 0..3 (forward exp(-i pi k / 4))
    zdbl t1 = INV ? zdbl{h * (o[1].re - o[1].im), h * (o[1].re + o[1].im)}
                  : zdbl{h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};
    zdbl t2 = rot90<INV>(o[2]);
    zdbl t3 = INV ? zdbl{-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im)}
                  : zdbl{h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im)};
    v[0] = zadd(e[0], o[0]);
    v[4] = zsub(e[0], o[0]);
    v[1] = zadd(e[1], t1);
    v[5] = zsub(e[1], t1);
    v[2] = zadd(e[2], t2);
    v[6] = zsub(e[2], t2);
    v[3] = zadd(e[3], t3);
    v[7] = zsub(e[3], t3);
}

// One Stockham autosort pass (Govindaraju et al., SC'08 formulation): with Ns
// the length already transformed, butterfly j reads x[j + r L/R], applies
// twiddle W_{Ns R}^{(j mod Ns) r}, does a radix-R DFT and writes
// y[(j/Ns) Ns R + (j mod Ns) + r Ns].  In place through registers.
template <int L, int R, bool INV>
__device__ inline void fft_pass(zdbl *buf, const zdbl *__restrict__ tw, int Ns) {
    constexpr int NB = L / R;
    constexpr int IT = (NB + 255) / 256;
    zdbl v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = threadIdx.x + 256 * it;
        if (j < NB) {
            const int jm = j % Ns;
            const int step = L / (Ns * R);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                zdbl x = buf[j + r * NB];
                if (r > 0 && jm > 0) {
                    zdbl w = tw[jm * r * step];
                    if (INV) w.im = -w.im;
                    x = zmul(x, w);
                }
                v[it][r] = x;
            }
            if (R == 8) dft8<INV>(v[it]);
            else if (R == 4) dft4<INV>(v[it]);
            else dft2<INV>(v[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int j = threadIdx.x + 256 * it;
        if (j < NB) {
            const int jm = j % Ns;
            const int base = (j / Ns) * Ns * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[it][r];
        }
    }
    __syncthreads();
}

template <int L, bool INV>
__device__ inline void fft(zdbl *buf, const zdbl *__restrict__ tw) {
    int Ns = 1;
    int rem = L;
    while (rem >= 8) {
        fft_pass<L, 8, INV>(buf, tw, Ns);
        Ns *= 8;
        rem /= 8;
    }
    if (rem == 4) fft_pass<L, 4, INV>(buf, tw, Ns);
    else if (rem == 2) fft_pass<L, 2, INV>(buf, tw, Ns);
}

// chi0 from the histogram.  Workgroup = one row mu and up to 16 consecutive
// nu >= mu.  Two real odd sequences a, b are packed as z = a + i b; since the
// DFT of a real odd sequence is i*alpha with alpha real, Z = i alpha - beta:
// alpha = Im Z, beta = -Re Z.  Then chi = IFFT(i alpha Kt) / L for each.
template <int L>
__global__ __launch_bounds__(256) void k_fftconv(int n, int n_omega, int nhb, const int64_t *__restrict__ H,
                                                 int64_t n_upper, const int32_t *__restrict__ s_dev,
                                                 const zdbl *__restrict__ Kt, const zdbl *__restrict__ tw,
                                                 zdbl *__restrict__ chi0) {
    __shared__ zdbl buf[L];
    __shared__ double rb[L];
    const int nch = (n + 15) / 16;
    const int mu = blockIdx.x / nch;
    const int nu0 = (blockIdx.x % nch) * 16;
    if (nu0 + 15 < mu) return;
    const int nua = max(nu0, mu), nue = min(nu0 + 16, n);
    const int s = *s_dev;
    const double inv_l = 1.0 / (double)L;
    const int64_t nn = (int64_t)n * n;
    const int64_t trow = (int64_t)mu * n - ((int64_t)mu * (mu - 1)) / 2 - mu;
    for (int va = nua; va < nue; va += 2) {
        const int vb = va + 1;
        const bool hasb = vb < nue;
        const int64_t ta = trow + va, tb = trow + vb;
        for (int q = threadIdx.x; q < L; q += 256) buf[q] = zdbl{0.0, 0.0};
        __syncthreads();
        for (int m = 1 + threadIdx.x; m < nhb; m += 256) {
            const double ha = ldexp((double)H[(int64_t)m * n_upper + ta], -s);
            const double hb = hasb ? ldexp((double)H[(int64_t)m * n_upper + tb], -s) : 0.0;
            buf[m] = zdbl{ha, hb};
            buf[L - m] = zdbl{-ha, -hb};
        }
        __syncthreads();
        fft<L, false>(buf, tw);
        for (int q = threadIdx.x; q < L; q += 256) {
            const zdbl Z = buf[q];
            const double al = Z.im;
            rb[q] = -Z.re;
            const zdbl K = Kt[q];
            buf[q] = zdbl{-al * K.im, al * K.re};
        }
        __syncthreads();
        fft<L, true>(buf, tw);
        for (int j = threadIdx.x; j < n_omega; j += 256) {
            const zdbl val = zdbl{buf[j].re * inv_l, buf[j].im * inv_l};
            chi0[j * nn + (int64_t)mu * n + va] = val;
            if (va != mu) chi0[j * nn + (int64_t)va * n + mu] = val;
        }
        if (hasb) {
            __syncthreads();
            for (int q = threadIdx.x; q < L; q += 256) {
                const double be = rb[q];
                const zdbl K = Kt[q];
                buf[q] = zdbl{-be * K.im, be * K.re};
            }
            __syncthreads();
            fft<L, true>(buf, tw);
            for (int j = threadIdx.x; j < n_omega; j += 256) {
                const zdbl val = zdbl{buf[j].re * inv_l, buf[j].im * inv_l};
                chi0[j * nn + (int64_t)mu * n + vb] = val;
                chi0[j * nn + (int64_t)vb * n + mu] = val;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_kspec(hipStream_t st, int n_omega, int j0, double domega, double eps, zdbl *Kt, zdbl *tw) {
    const int L = 2 * n_omega;
    hipLaunchKernelGGL(k_kspec, dim3((L + 255) / 256), dim3(256), 0, st, L, j0, domega, eps, Kt, tw);
    return hipGetLastError();
}

hipError_t launch_fftconv(hipStream_t st, int n, int n_omega, int nhb, const int64_t *H, const int32_t *s_dev,
                          const zdbl *Kt, const zdbl *tw, zdbl *chi0) {
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    const int nch = (n + 15) / 16;
    dim3 grid((unsigned)((int64_t)n * nch));
    const int L = 2 * n_omega;
    ProfScope ps(st, "fftconv", 0.0, 8.0 * nhb * (double)n_upper + 16.0 * n_omega * (double)n * n);
#define GW_FFT_CASE(LL)                                                                                    \
    case LL:                                                                                               \
        hipLaunchKernelGGL(k_fftconv<LL>, grid, dim3(256), 0, st, n, n_omega, nhb, H, n_upper, s_dev, Kt, tw, \
                           chi0);                                                                          \
        break;
    switch (L) {
        GW_FFT_CASE(32)
        GW_FFT_CASE(64)
        GW_FFT_CASE(128)
        GW_FFT_CASE(256)
        GW_FFT_CASE(512)
        GW_FFT_CASE(1024)
        GW_FFT_CASE(2048)
        GW_FFT_CASE(4096)
        default:
            return hipErrorInvalidValue;
    }
#undef GW_FFT_CASE
    return hipGetLastError();
}

}  // namespace gwk
