// chi0 from the histogram on gfx950: the Cauchy transform of the odd-extended
// spectral function as an FFT convolution with a precomputed kernel spectrum
// (Section 5.A eq. chi_by_spectra; Section 8.A does its convolutions by FFT).
#include "gw_internal.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

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
// Spectral bin value as a double: the exact histogram scaled by 2^-s, or a
// spectral array already in floating point.
__device__ inline double hval(const int64_t *H, int64_t i, int s) { return ldexp((double)H[i], -s); }
__device__ inline double hval(const double *H, int64_t i, int) { return H[i]; }

template <typename HT, int L>
__global__ __launch_bounds__(256) void k_fftconv(int n, int n_omega, int nhb, const HT *__restrict__ H,
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
    const int s = s_dev ? *s_dev : 0;
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
            const double ha = hval(H, (int64_t)m * n_upper + ta, s);
            const double hb = hasb ? hval(H, (int64_t)m * n_upper + tb, s) : 0.0;
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


// ------------------------------------------------------------------ wave FFT convolution
// One lane group of P = 64 NW lanes (NW waves) per (mu, nu) sequence, E = L / P
// complex values per lane kept in registers; a radix-R Stockham pass works on
// butterflies j = lane + P t (t < E / R), element r of butterfly t in register
// slot t R + r holding position j + (L / R) r.  Between passes the group
// exchanges through its own LDS region (real and imaginary parts in turn,
// positions padded by one double per 16 against bank conflicts); a single
// wave needs no workgroup barrier, a group of two waits at one.  The last
// pass leaves position q = lane + P sigma in the lane that also owns q in
// the first pass, so forward output, kernel multiply and inverse input stay
// in registers.  At L = 2048 two waves share a sequence (16 values per lane):
// one wave would need 32 and spill registers to scratch memory.
__device__ inline int fpad(int pos) { return pos + (pos >> 4); }

template <bool INV>
__device__ inline void dft16(zdbl *v) {
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    zdbl a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        a[n2][0] = v[n2];
        a[n2][1] = v[n2 + 4];
        a[n2][2] = v[n2 + 8];
        a[n2][3] = v[n2 + 12];
        dft4<INV>(a[n2]);
    }
    // twiddles W16^(n2 k1), forward exp(-2 pi i m / 16)
    const double wr[10] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1};
    const double wi[10] = {0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1};
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int m = n2 * k1;
            const zdbl w{wr[m], INV ? -wi[m] : wi[m]};
            a[n2][k1] = zmul(a[n2][k1], w);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        zdbl b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<INV>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <int R, bool INV>
__device__ inline void dftR(zdbl *v) {
    if constexpr (R == 16) dft16<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else dft2<INV>(v);
}

// Register slot of a butterfly element.  PERM: the data still sit in the
// last-pass layout of the forward transform (radix RL) while this pass reads
// them in the first-pass layout (radix R): canonical slot t R + r is position
// lane + 64 sg with sg = t + (E / R) r, which the forward transform left in
// slot (sg % (E / RL)) RL + sg / (E / RL).
template <int L, int R, int RL, bool PERM, int P = 64>
__device__ constexpr int wslot(int t, int r) {
    constexpr int E = L / P;
    if constexpr (!PERM) return t * R + r;
    const int sg = t + (E / R) * r;
    return (sg % (E / RL)) * RL + sg / (E / RL);
}

// Twiddle and butterfly of one pass (radix R, NS points already transformed).
template <int L, int R, int NS, bool INV, bool PERM = false, int RL = R, int P = 64>
__device__ inline void wpass(zdbl *x, const zdbl *__restrict__ tw, int lane) {
    constexpr int E = L / P, NBF = E / R;
#pragma unroll
    for (int t = 0; t < NBF; ++t) {
        const int j = lane + P * t;
        zdbl v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[wslot<L, R, RL, PERM, P>(t, r)];
        if constexpr (NS > 1) {
            // W^(jm r) for r < R from the table entries of r = 1, 2, 4, 8
            // (at most two further roundings per factor)
            const int jm = j & (NS - 1);
            constexpr int st = L / (NS * R);
            zdbl w[R];
            w[1] = tw[jm * st];
            if constexpr (R > 2) w[2] = tw[2 * jm * st];
            if constexpr (R > 4) w[4] = tw[4 * jm * st];
            if constexpr (R > 8) w[8] = tw[8 * jm * st];
            if constexpr (R > 2) w[3] = zmul(w[2], w[1]);
            if constexpr (R > 4) {
                w[5] = zmul(w[4], w[1]);
                w[6] = zmul(w[4], w[2]);
                w[7] = zmul(w[4], w[3]);
            }
            if constexpr (R > 8) {
#pragma unroll
                for (int r = 9; r < 16; ++r) w[r] = zmul(w[8], w[r - 8]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) {
                if (INV) w[r].im = -w[r].im;
                v[r] = zmul(v[r], w[r]);
            }
        }
        dftR<R, INV>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) x[wslot<L, R, RL, PERM, P>(t, r)] = v[r];
        __builtin_amdgcn_sched_barrier(0);  // one butterfly's registers at a time
    }
}

// Waits for the other waves of the lane group (P > 64: the whole workgroup,
// every wave of which runs the same passes).
template <int P>
__device__ inline void wsync() {
    if constexpr (P == 64) __builtin_amdgcn_wave_barrier();
    else __syncthreads();
}

// Outputs of a (R, NS) pass go to y = (j / NS) NS R + j % NS + r NS; the next
// pass (radix R2) reads position j2 + (L / R2) r2 into slot t2 R2 + r2.  All
// writes of a part precede its reads, so the reads may land in the same
// registers.
template <int L, int R, int NS, int R2, bool PERM = false, int RL = R, int P = 64>
__device__ inline void wexchange(zdbl *x, double *lds, int lane) {
    constexpr int E = L / P, NBF = E / R, NBF2 = E / R2;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int t = 0; t < NBF; ++t) {
            const int j = lane + P * t;
            const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const zdbl &v = x[wslot<L, R, RL, PERM, P>(t, r)];
                lds[fpad(base + r * NS)] = part ? v.im : v.re;
            }
        }
        wsync<P>();
#pragma unroll
        for (int t2 = 0; t2 < NBF2; ++t2)
#pragma unroll
            for (int r2 = 0; r2 < R2; ++r2) {
                const double d = lds[fpad(lane + P * t2 + (L / R2) * r2)];
                if (part) x[t2 * R2 + r2].im = d;
                else x[t2 * R2 + r2].re = d;
            }
        wsync<P>();
    }
}

// Whole FFT of length L in registers + the wave's LDS region; output in the
// layout of the last pass.  PERM: the input is in the last-pass layout (of a
// previous transform), else in the first-pass layout.
template <int L, bool INV, bool PERM, int P = 64>
__device__ inline void wfft(zdbl *x, double *lds, const zdbl *__restrict__ tw, int lane) {
    if constexpr (P == 128) {
        static_assert(L == 2048, "two waves per sequence only at L = 2048");
        wpass<L, 16, 1, INV, PERM, 8, P>(x, tw, lane);
        wexchange<L, 16, 1, 16, PERM, 8, P>(x, lds, lane);
        wpass<L, 16, 16, INV, false, 16, P>(x, tw, lane);
        wexchange<L, 16, 16, 8, false, 16, P>(x, lds, lane);
        wpass<L, 8, 256, INV, false, 8, P>(x, tw, lane);
    } else if constexpr (L == 2048) {
        wpass<L, 16, 1, INV, PERM, 8>(x, tw, lane);
        wexchange<L, 16, 1, 16, PERM, 8>(x, lds, lane);
        wpass<L, 16, 16, INV>(x, tw, lane);
        wexchange<L, 16, 16, 8>(x, lds, lane);
        wpass<L, 8, 256, INV>(x, tw, lane);
    } else if constexpr (L == 1024) {
        wpass<L, 16, 1, INV, PERM, 8>(x, tw, lane);
        wexchange<L, 16, 1, 8, PERM, 8>(x, lds, lane);
        wpass<L, 8, 16, INV>(x, tw, lane);
        wexchange<L, 8, 16, 8>(x, lds, lane);
        wpass<L, 8, 128, INV>(x, tw, lane);
    } else if constexpr (L == 512) {
        wpass<L, 8, 1, INV, PERM, 8>(x, tw, lane);
        wexchange<L, 8, 1, 8, PERM, 8>(x, lds, lane);
        wpass<L, 8, 8, INV>(x, tw, lane);
        wexchange<L, 8, 8, 8>(x, lds, lane);
        wpass<L, 8, 64, INV>(x, tw, lane);
    } else {
        static_assert(L == 256, "wave FFT length");
        wpass<L, 4, 1, INV, PERM, 4>(x, tw, lane);
        wexchange<L, 4, 1, 4, PERM, 4>(x, lds, lane);
        wpass<L, 4, 4, INV>(x, tw, lane);
        wexchange<L, 4, 4, 4>(x, lds, lane);
        wpass<L, 4, 16, INV>(x, tw, lane);
        wexchange<L, 4, 16, 4>(x, lds, lane);
        wpass<L, 4, 64, INV>(x, tw, lane);
    }
}

template <int L>
struct WPlan {
    static constexpr int R1 = (L == 2048 || L == 1024) ? 16 : (L == 512 ? 8 : 4);  // first pass radix
    static constexpr int RL = (L == 256) ? 4 : 8;                                  // last pass radix
    static constexpr int NW = (L == 2048) ? 2 : 1;                                 // waves per sequence
};

// chi0 from the histogram, one sequence per lane group.  Workgroup = 8 waves
// = row mu and SEQ = 8 / NW consecutive nu >= mu of one column group: the
// outputs are staged through LDS so that every SEQ lanes write SEQ * 16
// contiguous bytes of a chi0 row.  Each sequence: forward FFT of the odd
// extension (purely imaginary spectrum i alpha), times i Kt, inverse FFT,
// scale 1/L.  FULL: the spectral arrays are dense [m][n][n] (n_upper = n^2,
// every nu, no symmetry) and hold v a0, so the transform is v chi0 and the
// kernel writes A = 1 - v chi0.
template <typename HT, int L, bool FULL = false>
__global__ __launch_bounds__(512) void k_fftconv_w(int n, int n_omega, int nhb, const HT *__restrict__ H,
                                                   int64_t n_upper, const int32_t *__restrict__ s_dev,
                                                   const zdbl *__restrict__ Kt, const zdbl *__restrict__ tw,
                                                   zdbl *__restrict__ chi0) {
    constexpr int NW = WPlan<L>::NW, P = 64 * NW, SEQ = 8 / NW;
    constexpr int E = L / P, REG = L + L / 16;  // doubles per sequence region
    constexpr int R1 = WPlan<L>::R1, RL = WPlan<L>::RL;
    __shared__ double lds[SEQ * REG];
    const int nch = (n + SEQ - 1) / SEQ;
    const int mu = blockIdx.x / nch;
    const int nu0 = (blockIdx.x % nch) * SEQ;
    if (!FULL && nu0 + SEQ - 1 < mu) return;
    const int tid = threadIdx.x, lane = tid % P, w = tid / P;
    const int s = s_dev ? *s_dev : 0;
    const int64_t nn = (int64_t)n * n;
    const int64_t trow = FULL ? (int64_t)mu * n : (int64_t)mu * n - ((int64_t)mu * (mu - 1)) / 2 - mu;
    // histogram rows of the SEQ sequences, scaled to doubles: Hs[m][w], m < nhb
    double *Hs = lds;
    for (int idx = tid; idx < nhb * SEQ; idx += 512) {
        const int m = idx / SEQ, ww = idx % SEQ;
        const int nu = nu0 + ww;
        double v = 0.0;
        if (m >= 1 && (FULL || nu >= mu) && nu < n) v = hval(H, (int64_t)m * n_upper + trow + nu, s);
        Hs[m * (SEQ + 1) + ww] = v;
    }
    __syncthreads();
    // odd extension a(q) = h(q), a(L - q) = -h(q), in the first pass layout
    zdbl x[E];
#pragma unroll
    for (int t = 0; t < E / R1; ++t)
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int q = lane + P * t + (L / R1) * r;
            double a = 0.0;
            if (q < nhb) a = Hs[q * (SEQ + 1) + w];
            else if (q > L - nhb) a = -Hs[(L - q) * (SEQ + 1) + w];
            x[t * R1 + r] = zdbl{a, 0.0};
        }
    __syncthreads();
    double *my = lds + w * REG;
    wfft<L, false, false, P>(x, my, tw, lane);
    // times i Kt at position q = lane + P sg, in place in the last-pass layout
#pragma unroll
    for (int sg = 0; sg < E; ++sg) {
        const int sf = (sg % (E / RL)) * RL + sg / (E / RL);
        const zdbl K = Kt[lane + P * sg];
        const double al = x[sf].im;
        x[sf] = zdbl{-al * K.im, al * K.re};
        if ((sg & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // keep few loads in flight (registers)
    }
    wfft<L, true, true, P>(x, my, tw, lane);
    // stage q < n_omega (last-pass layout) as complex pairs in the sequence's region
    const double inv_l = 1.0 / (double)L;
#pragma unroll
    for (int sg = 0; sg < E / 2; ++sg) {
        const int sf = (sg % (E / RL)) * RL + sg / (E / RL);
        const int q = lane + P * sg;
        my[2 * q] = x[sf].re * inv_l;
        my[2 * q + 1] = x[sf].im * inv_l;
    }
    __syncthreads();
    for (int idx = tid; idx < SEQ * n_omega; idx += 512) {
        const int ww = idx % SEQ, j = idx / SEQ;
        const int nu = nu0 + ww;
        if ((FULL || nu >= mu) && nu < n) {
            const double *src = lds + ww * REG + 2 * j;
            zdbl v{src[0], src[1]};
            if (FULL) v = zdbl{(nu == mu ? 1.0 : 0.0) - v.re, -v.im};
            chi0[j * nn + (int64_t)mu * n + nu] = v;
        }
    }
}

// chi0 is symmetric: fill the strict lower triangle of every frequency from
// the upper one, 32 x 32 tiles through LDS (both sides coalesced rows).
// Workgroup = one upper tile (bi <= bj) for 8 consecutive frequencies.
__global__ __launch_bounds__(256) void k_symmetrize(int n, int n_omega, int nt, zdbl *__restrict__ chi0) {
    __shared__ zdbl t[32][33];
    int tile = blockIdx.x, bi = 0;
    while (tile >= nt - bi) {  // upper tiles enumerated row by row
        tile -= nt - bi;
        ++bi;
    }
    const int bj = bi + tile;
    const int64_t nn = (int64_t)n * n;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int j_end = min(n_omega, (int)(blockIdx.y + 1) * 8);
    for (int j = blockIdx.y * 8; j < j_end; ++j) {
        zdbl *c = chi0 + j * nn;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = bi * 32 + ty + 8 * q, col = bj * 32 + tx;
            if (r < n && col < n) t[ty + 8 * q][tx] = c[(int64_t)r * n + col];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = bj * 32 + ty + 8 * q, col = bi * 32 + tx;  // lower element (r, col) = upper (col, r)
            if (r < n && col < n && r > col) c[(int64_t)r * n + col] = t[tx][ty + 8 * q];
        }
        __syncthreads();
    }
}

// Bins m0 .. m0+cnt-1 of a packed spectral array as dense symmetric doubles,
// D[m - m0][mu][nu] = H[m][t(min, max)] (times 2^-s for the exact histogram);
// 32 x 32 tiles through LDS as in k_symmetrize.  Workgroup = one upper tile
// (bi <= bj) of bin m0 + blockIdx.y.
template <typename HT>
__global__ __launch_bounds__(256) void k_expand_bins(int n, int nt, const HT *__restrict__ H, int64_t n_upper,
                                                     const int32_t *__restrict__ s_dev, int m0,
                                                     double *__restrict__ D) {
    __shared__ double t[32][33];
    int tile = blockIdx.x, bi = 0;
    while (tile >= nt - bi) {
        tile -= nt - bi;
        ++bi;
    }
    const int bj = bi + tile;
    const int s = s_dev ? *s_dev : 0;
    const int64_t nn = (int64_t)n * n;
    const HT *Hm = H + ((int64_t)m0 + blockIdx.y) * n_upper;
    double *Dm = D + (int64_t)blockIdx.y * nn;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = bi * 32 + ty + 8 * q, c = bj * 32 + tx;
        double val = 0.0;
        if (r < n && c < n && c >= r) {
            const int64_t tr = (int64_t)r * n - ((int64_t)r * (r - 1)) / 2 - r;
            val = hval(Hm, tr + c, s);
            Dm[(int64_t)r * n + c] = val;
        }
        t[ty + 8 * q][tx] = val;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = bj * 32 + ty + 8 * q, c = bi * 32 + tx;  // lower (r, c) = upper (c, r)
        if (r < n && c < n && r > c) Dm[(int64_t)r * n + c] = t[tx][ty + 8 * q];
    }
}

}  // namespace

namespace {
template <typename HT>
hipError_t expand_bins_impl(hipStream_t st, int n, int m0, int cnt, const HT *H, int64_t n_upper,
                            const int32_t *s_dev, double *D) {
    if (cnt < 1) return hipSuccess;
    if (cnt > 65535 || m0 < 0) return hipErrorInvalidValue;
    const int nt = (n + 31) / 32;
    ProfScope pm(st, "expand_bins", 0.0, (8.0 * cnt) * ((double)n * (n + 1) / 2 + (double)n * n));
    hipLaunchKernelGGL((k_expand_bins<HT>), dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)cnt), dim3(256), 0, st, n,
                       nt, H, n_upper, s_dev, m0, D);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_expand_bins(hipStream_t st, int n, int m0, int cnt, const int64_t *H, int64_t n_upper,
                              const int32_t *s_dev, double *D) {
    return expand_bins_impl(st, n, m0, cnt, H, n_upper, s_dev, D);
}

hipError_t launch_expand_bins(hipStream_t st, int n, int m0, int cnt, const double *a, int64_t n_upper, double *D) {
    return expand_bins_impl(st, n, m0, cnt, a, n_upper, (const int32_t *)nullptr, D);
}

hipError_t launch_fftconv_A(hipStream_t st, int n, int n_omega, int nhb, const double *B, const zdbl *Kt,
                            const zdbl *tw, zdbl *A) {
    const int64_t nn = (int64_t)n * n;
    const int L = 2 * n_omega;
    ProfScope ps(st, "fftconv_A", 0.0, 8.0 * (nhb - 1) * (double)nn + 16.0 * n_omega * (double)nn);
    const int seq = L == 2048 ? 4 : 8;  // sequences per workgroup (two waves each at L = 2048)
    dim3 gw((unsigned)((int64_t)n * ((n + seq - 1) / seq)));
#define GW_FFTA_CASE(LL)                                                                                            \
    case LL:                                                                                                        \
        hipLaunchKernelGGL((k_fftconv_w<double, LL, true>), gw, dim3(512), 0, st, n, n_omega, nhb, B, nn,           \
                           (const int32_t *)nullptr, Kt, tw, A);                                                    \
        break;
    switch (L) {
        GW_FFTA_CASE(256)
        GW_FFTA_CASE(512)
        GW_FFTA_CASE(1024)
        GW_FFTA_CASE(2048)
        default:
            return hipErrorInvalidValue;
    }
#undef GW_FFTA_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ A route: Cauchy transform as a product
// The Cauchy transform of the odd-extended bins (Section 5.A eq.
// chi_by_spectra) at mesh point j is a fixed linear map of the bins, the same
// for every matrix entry:  sum_q T[j][q] x_q  with
//   T[j][q] = 1/(omega_j - q domega + i eps) - 1/(omega_j + q domega + i eps),
// omega_j = (j + j0) domega.  On the A route, with x_q = (v a0)_q and the
// identity in bin row 0 (bin 0 carries no weight in chi0), A = 1 - v chi0 is
// one complex-times-real product  A = -T' X  with T'[j][0] = -1.
// Rows of T': r = 0 is mesh point 0 (the lone point), r >= 1 is mesh point
// n_omega/2 + r - 1 (the solved half); ld = nhb.
__global__ void k_cauchy_T(int n_omega, int j0, double domega, double eps, int nhb, zdbl *__restrict__ T) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (q >= nhb) return;
    const int j = r == 0 ? 0 : n_omega / 2 + r - 1;
    zdbl t{-1.0, 0.0};
    if (q > 0) {
        const double xm = (double)(j + j0 - q) * domega, xp = (double)(j + j0 + q) * domega;
        const double dm = xm * xm + eps * eps, dp = xp * xp + eps * eps;
        t = zdbl{xm / dm - xp / dp, -eps / dm + eps / dp};
    }
    T[(int64_t)r * nhb + q] = t;
}

// Bin row 0 of X set to the identity pattern (X[0][mu][nu] = delta_{mu nu}).
__global__ void k_eye_row(int n, int64_t nn, double *__restrict__ X0) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x)
        X0[e] = (e % (n + 1) == 0) ? 1.0 : 0.0;
}

// The lone mesh point j = 0 (no mirror partner, one row of the product):
// A[0][e] = -sum_q T'[0][q] X[q][e], one entry per thread, rows of X read
// coalesced.
__global__ __launch_bounds__(256) void k_cauchy_row0(int64_t nn, int nhb, const zdbl *__restrict__ T0,
                                                     const double *__restrict__ X, zdbl *__restrict__ A0) {
    extern __shared__ zdbl t0[];
    for (int q = threadIdx.x; q < nhb; q += blockDim.x) t0[q] = T0[q];
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < nhb; ++q) {
        const double x = X[(int64_t)q * nn + e];
        re = fma(t0[q].re, x, re);
        im = fma(t0[q].im, x, im);
    }
    A0[e] = zdbl{-re, -im};
}

hipError_t launch_cauchy_A(hipStream_t st, int n, int n_omega, int nhb, int j0, double domega, double eps,
                           double *X, zdbl *T, zdbl *A) {
    const int64_t nn = (int64_t)n * n;
    const int half = n_omega / 2;
    hipLaunchKernelGGL(k_cauchy_T, dim3((nhb + 255) / 256, half + 1), dim3(256), 0, st, n_omega, j0, domega, eps, nhb,
                       T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>((nn + 255) / 256, 16384);
    hipLaunchKernelGGL(k_eye_row, dim3((unsigned)blocks), dim3(256), 0, st, n, nn, X);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the solved half j = n_omega/2 .. n_omega-1 in one product, which also
    // writes the other half by A(-omega) = A(omega)* (v real)
    if ((e = launch_zdgemm_wide(st, half, (int)nn, nhb, -1.0, T + nhb, nhb, X, nn, A + (int64_t)half * nn, nn,
                                true)) != hipSuccess)
        return e;
    {
        ProfScope ps(st, "cauchy_row0", 4.0 * (double)nn * nhb, 8.0 * (double)nn * nhb + 16.0 * (double)nn);
        hipLaunchKernelGGL(k_cauchy_row0, dim3((unsigned)((nn + 255) / 256)), dim3(256), sizeof(zdbl) * nhb, st, nn,
                           nhb, T, X, A);
        return hipGetLastError();
    }
}

hipError_t launch_kspec(hipStream_t st, int n_omega, int j0, double domega, double eps, zdbl *Kt, zdbl *tw) {
    const int L = 2 * n_omega;
    hipLaunchKernelGGL(k_kspec, dim3((L + 255) / 256), dim3(256), 0, st, L, j0, domega, eps, Kt, tw);
    return hipGetLastError();
}

hipError_t launch_symmetrize(hipStream_t st, int n, int n_omega, zdbl *chi0) {
    const int nt = (n + 31) / 32;
    ProfScope pm(st, "symmetrize", 0.0, 16.0 * 2.0 * n_omega * ((double)n * (n - 1) / 2));
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)((n_omega + 7) / 8)), dim3(256), 0,
                       st, n, n_omega, nt, chi0);
    return hipGetLastError();
}

namespace {
template <typename HT>
hipError_t fftconv_impl(hipStream_t st, int n, int n_omega, int nhb, const HT *H, const int32_t *s_dev,
                        const zdbl *Kt, const zdbl *tw, zdbl *chi0, bool symmetrize) {
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    const int L = 2 * n_omega;
    if (L >= 256 && L <= 2048) {
        // wave kernel on the upper triangle, then the lower one by symmetry
        {
            ProfScope ps(st, "fftconv", 0.0, 8.0 * nhb * (double)n_upper + 16.0 * n_omega * (double)n_upper);
            const int seq = L == 2048 ? 4 : 8;  // sequences per workgroup (two waves each at L = 2048)
            dim3 gw((unsigned)((int64_t)n * ((n + seq - 1) / seq)));
#define GW_FFTW_CASE(LL)                                                                                     \
    case LL:                                                                                                 \
        hipLaunchKernelGGL((k_fftconv_w<HT, LL>), gw, dim3(512), 0, st, n, n_omega, nhb, H, n_upper, s_dev, Kt, tw, \
                           chi0);                                                                            \
        break;
            switch (L) {
                GW_FFTW_CASE(256)
                GW_FFTW_CASE(512)
                GW_FFTW_CASE(1024)
                GW_FFTW_CASE(2048)
            }
#undef GW_FFTW_CASE
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return symmetrize ? launch_symmetrize(st, n, n_omega, chi0) : hipSuccess;
    }
    ProfScope ps(st, "fftconv", 0.0, 8.0 * nhb * (double)n_upper + 16.0 * n_omega * (double)n * n);
    const int nch = (n + 15) / 16;
    dim3 grid((unsigned)((int64_t)n * nch));
#define GW_FFT_CASE(LL)                                                                                    \
    case LL:                                                                                               \
        hipLaunchKernelGGL((k_fftconv<HT, LL>), grid, dim3(256), 0, st, n, n_omega, nhb, H, n_upper, s_dev, Kt, tw, \
                           chi0);                                                                          \
        break;
    switch (L) {
        GW_FFT_CASE(32)
        GW_FFT_CASE(64)
        GW_FFT_CASE(128)
        GW_FFT_CASE(4096)
        default:
            return hipErrorInvalidValue;
    }
#undef GW_FFT_CASE
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fftconv(hipStream_t st, int n, int n_omega, int nhb, const int64_t *H, const int32_t *s_dev,
                          const zdbl *Kt, const zdbl *tw, zdbl *chi0, bool symmetrize) {
    return fftconv_impl(st, n, n_omega, nhb, H, s_dev, Kt, tw, chi0, symmetrize);
}

hipError_t launch_fftconv(hipStream_t st, int n, int n_omega, int nhb, const double *A, const zdbl *Kt,
                          const zdbl *tw, zdbl *chi0, bool symmetrize) {
    return fftconv_impl(st, n, n_omega, nhb, A, (const int32_t *)nullptr, Kt, tw, chi0, symmetrize);
}

namespace {

// K[j][m - m_lo] = 1/(w_j - m d + i eps) - 1/(w_j + m d + i eps), w_j = w0 + j dw
__global__ void k_cauchy_table(int n_om, double w0, double dw, int nhb, int m_lo, double d, double eps, zdbl *K) {
    const int M = nhb - m_lo;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_om * M) return;
    const int j = idx / M, m = m_lo + idx % M;
    const double w = w0 + j * dw, sm = m * d;
    const double a = w - sm, b = w + sm, e2 = eps * eps;
    const double da = a * a + e2, db = b * b + e2;
    // 1/(a + i eps) = (a - i eps) / (a^2 + eps^2)
    K[idx] = zdbl{a / da - b / db, -eps / da + eps / db};
}

// chi[j][mu][nu] += sum_m 2^-s H[m][mu<=nu] K[j][m - m_lo] on the upper
// triangle, one packed (mu <= nu) per thread.  Row m_lo is read from H_lo when
// that is given.  K is uniform over the workgroup (scalar loads); each thread
// keeps CJ frequencies in registers and walks its histogram column once per
// chunk of frequencies.
constexpr int CJ = 16;
__global__ __launch_bounds__(256) void k_cauchy_add(int n, int n_om, int nhb, int m_lo, const int64_t *__restrict__ H,
                                                    const int64_t *__restrict__ H_lo, const int32_t *__restrict__ s_dev,
                                                    const zdbl *__restrict__ K, zdbl *__restrict__ chi) {
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_upper) return;
    // row mu of the packed upper triangle: r(mu) = mu n - mu (mu - 1) / 2 <= t < r(mu + 1)
    auto rstart = [&](int64_t r) { return r * n - (r * (r - 1)) / 2; };
    const double b2 = 2.0 * n + 1.0;
    int64_t mu = (int64_t)((b2 - sqrt(b2 * b2 - 8.0 * (double)t)) * 0.5);
    if (mu < 0) mu = 0;
    if (mu > n - 1) mu = n - 1;
    while (mu > 0 && rstart(mu) > t) --mu;
    while (mu < n - 1 && rstart(mu + 1) <= t) ++mu;
    const int64_t nu = mu + (t - rstart(mu));
    const int s = *s_dev;
    const int M = nhb - m_lo;
    const int64_t nn = (int64_t)n * n;
    for (int j0 = 0; j0 < n_om; j0 += CJ) {
        const int nj = min(CJ, n_om - j0);
        double ar[CJ], ai[CJ];
#pragma unroll
        for (int q = 0; q < CJ; ++q) ar[q] = ai[q] = 0.0;
        for (int mm = 0; mm < M; ++mm) {
            const int64_t hv = (mm == 0 && H_lo) ? H_lo[t] : H[(int64_t)(m_lo + mm) * n_upper + t];
            const double h = ldexp((double)hv, -s);
            const zdbl *Kc = K + (int64_t)j0 * M + mm;
#pragma unroll
            for (int q = 0; q < CJ; ++q)
                if (q < nj) {
                    const zdbl k = Kc[(int64_t)q * M];
                    ar[q] += h * k.re;
                    ai[q] += h * k.im;
                }
        }
#pragma unroll
        for (int q = 0; q < CJ; ++q)
            if (q < nj) {
                zdbl *c = chi + (int64_t)(j0 + q) * nn + mu * n + nu;
                zdbl v = *c;
                v.re += ar[q];
                v.im += ai[q];
                *c = v;
            }
    }
}

}  // namespace

hipError_t launch_cauchy_table(hipStream_t st, int n_om, double w0, double dw, int nhb, int m_lo, double d,
                               double eps, zdbl *K) {
    const int64_t total = (int64_t)n_om * (nhb - m_lo);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cauchy_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n_om, w0, dw, nhb,
                       m_lo, d, eps, K);
    return hipGetLastError();
}

hipError_t launch_cauchy_add(hipStream_t st, int n, int n_om, int nhb, int m_lo, const int64_t *H,
                             const int64_t *H_lo, const int32_t *s_dev, const zdbl *K, zdbl *chi) {
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    if (nhb - m_lo <= 0 || n_om <= 0 || n_upper == 0) return hipSuccess;
    ProfScope ps(st, "cauchy_add", 8.0 * (nhb - m_lo) * (double)n_om * n_upper,
                 8.0 * (nhb - m_lo) * (double)n_upper + 32.0 * n_om * (double)n_upper);
    hipLaunchKernelGGL(k_cauchy_add, dim3((unsigned)((n_upper + 255) / 256)), dim3(256), 0, st, n, n_om, nhb, m_lo, H,
                       H_lo, s_dev, K, chi);
    return hipGetLastError();
}

}  // namespace gwk
