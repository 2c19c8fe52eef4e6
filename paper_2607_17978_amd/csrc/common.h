// Device-side building blocks shared by the kernels of the particle-mesh QEq
// library: complex arithmetic, cardinal B-splines, the LDS-resident mixed-radix
// Stockham FFT and block reductions in FP64.  gfx950 only (64-wide waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#define QEQ_MAXP 8          // largest supported spline order
#define QEQ_FFT_MAXST 10    // largest number of radix stages
#define QEQ_FFT_EMAX 40     // complex elements one thread holds during a stage

// ---------------------------------------------------------------------------
// complex helpers (float2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 cmul_mi(float2 a, bool inv) {
    return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Cardinal B-splines (Essmann et al. smooth PME; the paper's PPPM solver).
// For an atom at grid coordinate u with base h = floor(u), w = u - h, grid
// point h - k (k = 0..p-1) gets weight M_p(w + k).  The recursion
//   M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1),  M_2(x) = 1 - |x - 1|
// is evaluated on the p shifted arguments at once; the derivative is
//   M_n'(x) = M_{n-1}(x) - M_{n-1}(x - 1).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void bspline_weights(T w, int p, T* c, T* dc) {
    T prev[QEQ_MAXP];
    c[0] = w;
    c[1] = T(1) - w;
#pragma unroll
    for (int k = 2; k < QEQ_MAXP; ++k) c[k] = T(0);
    for (int n = 3; n <= p; ++n) {
        if (n == p) {
            for (int k = 0; k < QEQ_MAXP; ++k) prev[k] = c[k];
        }
        T inv = T(1) / T(n - 1);
        // c_n[k] = ((w+k) c[k] + (n - w - k) c[k-1]) / (n-1), descending k
        for (int k = n - 1; k >= 1; --k)
            c[k] = ((w + T(k)) * c[k] + (T(n) - w - T(k)) * c[k - 1]) * inv;
        c[0] = w * c[0] * inv;
    }
    if (p == 2) {
        prev[0] = T(1);
        for (int k = 1; k < QEQ_MAXP; ++k) prev[k] = T(0);
    }
    dc[0] = prev[0];
    for (int k = 1; k < p; ++k) dc[k] = prev[k] - prev[k - 1];
}

// ---------------------------------------------------------------------------
// FFT plan for one axis length K = 2^a 3^b 5^c: radix list and twiddles
// W_K^j = exp(-2 pi i j / K) (computed in FP64 on the host, stored FP32).
// ---------------------------------------------------------------------------
struct FftAxis {
    int K;
    int nst;
    int radix[QEQ_FFT_MAXST];
    const float2* tw;   // device table, K entries
};

// Small DFTs: X[k] = sum_n x[n] W^{nk}, W = exp(-+ 2 pi i / R) (forward / inverse).
template <int R> __device__ __forceinline__ void dft(float2* v, bool inv);

template <> __device__ __forceinline__ void dft<2>(float2* v, bool) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void dft<3>(float2* v, bool inv) {
    const float c1 = -0.5f, s1 = 0.86602540378443864676f;
    float2 a = v[0], b = v[1], c = v[2];
    float2 sbc = cadd(b, c), dbc = csub(b, c);
    float2 t = make_float2(a.x + c1 * sbc.x, a.y + c1 * sbc.y);
    float2 u = cmul_mi(cscale(dbc, s1), inv);   // -i s1 (b - c) forward
    v[0] = cadd(a, sbc);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <> __device__ __forceinline__ void dft<4>(float2* v, bool inv) {
    float2 a = v[0], b = v[1], c = v[2], d = v[3];
    float2 s0 = cadd(a, c), d0 = csub(a, c);
    float2 s1 = cadd(b, d), d1 = cmul_mi(csub(b, d), inv);
    v[0] = cadd(s0, s1);
    v[2] = csub(s0, s1);
    v[1] = cadd(d0, d1);
    v[3] = csub(d0, d1);
}

template <> __device__ __forceinline__ void dft<5>(float2* v, bool inv) {
    // cos / sin of 2 pi / 5 and 4 pi / 5
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    float2 a = v[0];
    float2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    float2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    float2 t1 = make_float2(a.x + c1 * p1.x + c2 * p2.x, a.y + c1 * p1.y + c2 * p2.y);
    float2 t2 = make_float2(a.x + c2 * p1.x + c1 * p2.x, a.y + c2 * p1.y + c1 * p2.y);
    // forward: X1 = t1 - i (s1 m1 + s2 m2), X2 = t2 - i (s2 m1 - s1 m2)
    float2 u1 = cmul_mi(make_float2(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y), inv);
    float2 u2 = cmul_mi(make_float2(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y), inv);
    v[0] = make_float2(a.x + p1.x + p2.x, a.y + p1.y + p2.y);
    v[1] = cadd(t1, u1);
    v[4] = csub(t1, u1);
    v[2] = cadd(t2, u2);
    v[3] = csub(t2, u2);
}

template <> __device__ __forceinline__ void dft<8>(float2* v, bool inv) {
    const float h = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e, inv);
    dft<4>(o, inv);
    // W8^k o[k], W8 = exp(-+ i pi / 4)
    float2 w1 = inv ? make_float2(h, h) : make_float2(h, -h);
    float2 w3 = inv ? make_float2(-h, h) : make_float2(-h, -h);
    o[1] = cmul(o[1], w1);
    o[2] = cmul_mi(o[2], inv);
    o[3] = cmul(o[3], w3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

// ---------------------------------------------------------------------------
// Composite small DFTs (radix 6, 10, 12, 16, 20) in registers: for
// N = R1 R2, n = R2 n1 + n2 and k = k1 + R1 k2,
//   X[k1 + R1 k2] = sum_n2 W_R2^{n2 k2} W_N^{n2 k1} (sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}),
// i.e. R2 DFTs of length R1, constant twiddles W_N^{n2 k1}, R1 DFTs of
// length R2.  A radix-16 stage does in one LDS pass what two radix-4
// stages do in two.
// ---------------------------------------------------------------------------
template <int... I, typename F>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// cos and sin of 2 pi m / N at compile time (Taylor series after reduction
// to [-pi/4, pi/4] by octant; double precision, rounded once to float)
constexpr double ce_sin_series(double x) {
    double t = x, s = x;
    for (int k = 1; k < 16; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double ce_cos_series(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 16; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
// angle 2 pi m / N written as (octant o, remainder r) with 8 m = o N + r,
// 0 <= r < N: theta = o pi / 4 + 2 pi r / (8 N)
constexpr double ce_trig(int m, int N, bool want_sin) {
    const int mm = ((m % N) + N) % N;
    const int o = (8 * mm) / N, r = 8 * mm - o * N;
    const double x = 2.0 * 3.14159265358979323846 * r / (8.0 * N);   // [0, pi/4)
    const double h = 0.70710678118654752440;
    // cos / sin of o pi / 4 + x from those of x
    const double cx = ce_cos_series(x), sx = ce_sin_series(x);
    const double co[8] = {1, h, 0, -h, -1, -h, 0, h};
    const double so[8] = {0, h, 1, h, 0, -h, -1, -h};
    return want_sin ? so[o] * cx + co[o] * sx : co[o] * cx - so[o] * sx;
}

// x W_N^M, W_N = exp(-+ 2 pi i / N): multiples of pi / 2 by sign changes and
// swaps, the others by one complex product with constant factors
template <int N, int M>
__device__ __forceinline__ float2 twiddle_const(float2 x, bool inv) {
    constexpr int m = M % N;
    if constexpr (m == 0) {
        return x;
    } else if constexpr (4 * m == N) {
        return cmul_mi(x, inv);
    } else if constexpr (2 * m == N) {
        return make_float2(-x.x, -x.y);
    } else if constexpr (4 * m == 3 * N) {
        return cmul_mi(x, !inv);
    } else {
        constexpr float c = (float)ce_trig(m, N, false), sn = (float)ce_trig(m, N, true);
        return cmul(x, make_float2(c, inv ? sn : -sn));
    }
}

template <int R1, int R2>
__device__ __forceinline__ void dft_ct2(float2* v, bool inv) {
    constexpr int N = R1 * R2;
    float2 t[N];
    static_for<R2>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        float2 a[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[R2 * n1 + n2];
        dft<R1>(a, inv);
        static_for<R1>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            t[n2 * R1 + k1] = twiddle_const<N, n2 * k1>(a[k1], inv);
        });
    });
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        float2 b[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) b[n2] = t[n2 * R1 + k1];
        dft<R2>(b, inv);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
    }
}

template <> __device__ __forceinline__ void dft<6>(float2* v, bool inv) { dft_ct2<3, 2>(v, inv); }
template <> __device__ __forceinline__ void dft<10>(float2* v, bool inv) { dft_ct2<5, 2>(v, inv); }
template <> __device__ __forceinline__ void dft<12>(float2* v, bool inv) { dft_ct2<4, 3>(v, inv); }
template <> __device__ __forceinline__ void dft<16>(float2* v, bool inv) { dft_ct2<4, 4>(v, inv); }
template <> __device__ __forceinline__ void dft<20>(float2* v, bool inv) { dft_ct2<5, 4>(v, inv); }

// One Stockham (decimation-in-time, self-sorting) stage of radix R on ncol
// interleaved columns held in LDS: element (index k, column c) lives at
// buf[k * ncol + c].  Each butterfly j of a column reads x[j + r K/R],
// applies the twiddles W_{Ns R}^{(j mod Ns) r}, does a length-R DFT and writes
// y[(j / Ns) Ns R + (j mod Ns) + r Ns].  The stage is done in place: all reads
// go to registers before a barrier, then all writes.
template <int R>
__device__ __forceinline__ void fft_stage(float2* buf, int K, int Ns, int ncol_log2,
                                          const float2* tw, bool inv, int tid, int nthr) {
    constexpr int MAXIT = (QEQ_FFT_EMAX + R - 1) / R;
    const int per = K / R;
    const int ncol = 1 << ncol_log2;
    const int nitems = per * ncol;
    const int step = K / (Ns * R);
    float2 v[MAXIT][R];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        int item = tid + it * nthr;
        if (item < nitems) {
            int c = item & (ncol - 1), j = item >> ncol_log2;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = buf[(j + r * per) * ncol + c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        int item = tid + it * nthr;
        if (item < nitems) {
            int c = item & (ncol - 1), j = item >> ncol_log2;
            int k = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[k * r * step];
                if (inv) w.y = -w.y;
                v[it][r] = cmul(v[it][r], w);
            }
            dft<R>(v[it], inv);
            int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(base + r * Ns) * ncol + c] = v[it][r];
        }
    }
    __syncthreads();
}

// Full length-K transform of ncol columns in LDS (unnormalised both ways).
__device__ __forceinline__ void fft_lds(float2* buf, const FftAxis& ax, int ncol_log2,
                                        const float2* tw_lds, bool inv, int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < ax.nst; ++s) {
        int R = ax.radix[s];
        switch (R) {
            case 2: fft_stage<2>(buf, ax.K, Ns, ncol_log2, tw_lds, inv, tid, nthr); break;
            case 3: fft_stage<3>(buf, ax.K, Ns, ncol_log2, tw_lds, inv, tid, nthr); break;
            case 4: fft_stage<4>(buf, ax.K, Ns, ncol_log2, tw_lds, inv, tid, nthr); break;
            case 5: fft_stage<5>(buf, ax.K, Ns, ncol_log2, tw_lds, inv, tid, nthr); break;
            default: fft_stage<8>(buf, ax.K, Ns, ncol_log2, tw_lds, inv, tid, nthr); break;
        }
        Ns *= R;
    }
}

// ---------------------------------------------------------------------------
// The same Stockham transform with the length, the radix sequence, the column
// count, the LDS row stride and the thread count fixed at compile time: every
// index computation folds to shifts and multiplications by constants, only
// the radices the length needs are instantiated, and register arrays are
// sized exactly.  Element (k, c) lives at buf[k * KS + c * CS].
// ---------------------------------------------------------------------------
// Stage radices of a compile-time length.  Composite plan: the fewest stages
// (one LDS pass each) over the radices 2, 3, 4, 5, 8 and the register
// composites 6, 10, 12, 16, 20; among those the smallest largest radix;
// larger radices first (192 = 16 x 12, 96 = 12 x 8, 320 = 20 x 16).
// Lengths that need more than three such stages, and the plain plan, take
// 5s, 3s, 8s, then 4 or 2 (192 = 3 x 8 x 8).
constexpr bool ct_radix_ok(int r) {
    return r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 8 || r == 10 || r == 12 || r == 16 || r == 20;
}
constexpr int ct_radix_plan(int K, int s, bool composite) {
    if (!composite) {
        int n = K, idx = 0;
        while (n % 5 == 0) { if (idx == s) return 5; n /= 5; ++idx; }
        while (n % 3 == 0) { if (idx == s) return 3; n /= 3; ++idx; }
        while (n % 8 == 0) { if (idx == s) return 8; n /= 8; ++idx; }
        if (n == 4) { if (idx == s) return 4; n = 1; ++idx; }
        if (n == 2) { if (idx == s) return 2; n = 1; ++idx; }
        return 0;
    }
    if (ct_radix_ok(K)) return s == 0 ? K : 0;
    int b1 = 0, b2 = 0, b3 = 0, best = 1 << 30;
    for (int a = 20; a >= 2; --a) {
        if (!ct_radix_ok(a) || K % a) continue;
        const int c = K / a;
        if (ct_radix_ok(c) && a >= c && a < best) { best = a; b1 = a; b2 = c; }
    }
    if (b1) return s == 0 ? b1 : (s == 1 ? b2 : 0);
    for (int a = 20; a >= 2; --a) {
        if (!ct_radix_ok(a) || K % a) continue;
        for (int b = a; b >= 2; --b) {
            if (!ct_radix_ok(b) || (K / a) % b) continue;
            const int c = K / a / b;
            if (ct_radix_ok(c) && b >= c && a < best) { best = a; b1 = a; b2 = b; b3 = c; }
        }
    }
    if (b1) return s == 0 ? b1 : (s == 1 ? b2 : (s == 2 ? b3 : 0));
    return ct_radix_plan(K, s, false);
}
// The composite plan is taken while each of its stages still gives every
// other thread of the block a butterfly ((K / R) ncol >= nthr / 2): on
// narrow tiles (320^3 rows of 4 or 8 columns) the few large butterflies
// leave most of the block idle and the plain plan is faster.
constexpr bool ct_composite(int K, int ncol, int nthr) {
    for (int s = 0; ct_radix_plan(K, s, true) != 0; ++s)
        if ((K / ct_radix_plan(K, s, true)) * ncol * 2 < nthr) return false;
    return true;
}
constexpr int ct_radix_at(int K, int s, int ncol, int nthr) {
    return ct_radix_plan(K, s, ct_composite(K, ncol, nthr));
}

template <int K, int R, int NS, int NCOL, int KS, int NTHR, bool INV, int CS = 1>
__device__ __forceinline__ void fft_stage_ct(float2* buf, const float2* tw, int tid) {
    constexpr int PER = K / R;
    constexpr int NITEMS = PER * NCOL;
    constexpr int IT = (NITEMS + NTHR - 1) / NTHR;
    constexpr int STEP = K / (NS * R);
    float2 v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int item = tid + it * NTHR;
        if (NITEMS % NTHR == 0 || item < NITEMS) {
            const int c = item % NCOL, j = item / NCOL;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = buf[(j + r * PER) * KS + c * CS];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int item = tid + it * NTHR;
        if (NITEMS % NTHR == 0 || item < NITEMS) {
            const int c = item % NCOL, j = item / NCOL;
            const int kk = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[kk * r * STEP];
                    if (INV) w.y = -w.y;
                    v[it][r] = cmul(v[it][r], w);
                }
            }
            dft<R>(v[it], INV);
            const int base = (j - kk) * R + kk;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(base + r * NS) * KS + c * CS] = v[it][r];
        }
    }
    __syncthreads();
}

// CS: stride between columns (1 = interleaved columns; a transposed layout
// has KS = 1 and CS = the row length).
// SEND: the stage to stop before (the transform's remaining stages can then
// be done by the caller, e.g. one that stores straight to global memory).
template <int K, int NCOL, int KS, int NTHR, bool INV, int S = 0, int NS = 1, int CS = 1, int SEND = 64>
__device__ __forceinline__ void fft_ct(float2* buf, const float2* tw, int tid) {
    constexpr int R = ct_radix_at(K, S, NCOL, NTHR);
    if constexpr (R != 0 && S < SEND) {
        fft_stage_ct<K, R, NS, NCOL, KS, NTHR, INV, CS>(buf, tw, tid);
        fft_ct<K, NCOL, KS, NTHR, INV, S + 1, NS * R, CS, SEND>(buf, tw, tid);
    }
}

// Number of radix stages of the compile-time transform of length K on ncol
// columns with nthr threads, and the product of the radices before stage s.
constexpr int ct_nstages(int K, int ncol, int nthr) {
    int s = 0;
    while (ct_radix_at(K, s, ncol, nthr) != 0) ++s;
    return s;
}
constexpr int ct_span(int K, int s, int ncol, int nthr) {
    int ns = 1;
    for (int t = 0; t < s; ++t) ns *= ct_radix_at(K, t, ncol, nthr);
    return ns;
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8), and each XCD has its own L2.  Renumbering the blocks so that the
// blocks of one XCD cover one contiguous range of work keeps neighbouring
// tiles or atoms, which read the same cache lines, in the same L2.  A
// bijection of [0, nb) for any nb.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int x = b & 7, j = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + j;
}

// ---------------------------------------------------------------------------
// Global -> LDS staging.  A strided copy loop waits for each load before its
// LDS store, so a thread's loads run one memory round trip apart; these
// helpers issue all of a thread's loads into registers first and store them
// afterwards, so the whole copy costs one round trip.  ld(t) returns element
// t, st(t, v) stores it; COUNT known at compile time (every load in flight at
// once) or at run time (CH loads in flight per step).
// ---------------------------------------------------------------------------
template <int COUNT, int NTH, typename T, typename Ld, typename St>
__device__ __forceinline__ void stage_ct(int tid, Ld ld, St st) {
    constexpr int PER = (COUNT + NTH - 1) / NTH;
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid + u * NTH;
        if (COUNT % NTH == 0 || t < COUNT) v[u] = ld(t);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid + u * NTH;
        if (COUNT % NTH == 0 || t < COUNT) st(t, v[u]);
    }
}

// Two arrays in one round trip (e.g. a twiddle table and a data tile).
template <int C1, int C2, int NTH, typename T, typename Ld1, typename St1, typename Ld2, typename St2>
__device__ __forceinline__ void stage2_ct(int tid, Ld1 ld1, St1 st1, Ld2 ld2, St2 st2) {
    constexpr int P1 = (C1 + NTH - 1) / NTH, P2 = (C2 + NTH - 1) / NTH;
    T a[P1], b[P2];
#pragma unroll
    for (int u = 0; u < P1; ++u) {
        const int t = tid + u * NTH;
        if (C1 % NTH == 0 || t < C1) a[u] = ld1(t);
    }
#pragma unroll
    for (int u = 0; u < P2; ++u) {
        const int t = tid + u * NTH;
        if (C2 % NTH == 0 || t < C2) b[u] = ld2(t);
    }
#pragma unroll
    for (int u = 0; u < P1; ++u) {
        const int t = tid + u * NTH;
        if (C1 % NTH == 0 || t < C1) st1(t, a[u]);
    }
#pragma unroll
    for (int u = 0; u < P2; ++u) {
        const int t = tid + u * NTH;
        if (C2 % NTH == 0 || t < C2) st2(t, b[u]);
    }
}

template <int CH, typename T, typename Ld, typename St>
__device__ __forceinline__ void stage_rt(int count, int tid, int nth, Ld ld, St st) {
    for (int t0 = tid; t0 < count; t0 += CH * nth) {
        T v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int t = t0 + u * nth;
            if (t < count) v[u] = ld(t);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int t = t0 + u * nth;
            if (t < count) st(t, v[u]);
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 block reductions (wave64 shuffles, then LDS across waves)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the block; result valid in thread 0.  blockDim <= 1024.
template <int NV>
__device__ __forceinline__ void block_sum(double* v) {
    __shared__ double red[16][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wid][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += red[w][k];
        }
    }
    __syncthreads();
}

// Every thread of the block obtains the totals of NV per-block partial sums
// laid out as part[b * NV + k], b < nparts.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* part, int nparts, double* out) {
    __shared__ double tot[NV];
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += part[b * NV + k];
    }
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = tot[k];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Real-space pair kernel K(r) = [erf(r/(sqrt2 gamma)) - erf(r/(sqrt2 eta))]/r
// (the erfc-difference of the Ewald split for Gaussian charges, SI "Ewald
// Summation"), gamma = sqrt(sigma_i^2 + sigma_j^2), and K'(r)/r for forces.
// A series replaces the quotient below r = 1e-4 bohr.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_kernel(double r, double gam, double eta, double* K, double* dKr) {
    const double two_sqrtpi = 1.12837916709551257390;
    double a = 0.70710678118654752440 / gam, b = 0.70710678118654752440 / eta;
    if (r < 1e-4) {
        *K = two_sqrtpi * ((a - b) - (a * a * a - b * b * b) * r * r / 3.0);
        *dKr = -two_sqrtpi * 2.0 * (a * a * a - b * b * b) / 3.0;
        return;
    }
    double e = erf(a * r) - erf(b * r);
    double kv = e / r;
    double d = (two_sqrtpi * (a * exp(-a * a * r * r) - b * exp(-b * b * r * r)) - kv) / r;
    *K = kv;
    *dKr = d / r;
}

// ---------------------------------------------------------------------------
// Mesh self-interaction of one atom.  The mesh reproduces the reciprocal self
// term of atom i as theta_i^T Theta theta_i, which depends on where the atom
// sits inside its grid cell.  With separable spline weights W_a,
//   theta_i^T Theta theta_i = sum_d Theta(d) R_1(d_1) R_2(d_2) R_3(d_3),
//   R_a(d) = sum_{k' - k = d} W_a[k] W_a[k'],  |d_a| <= p - 1,
// where tab holds Theta(d) on the (2p-1)^3 offsets (d_1 slowest).  Returns the
// value and its derivative with respect to the grid coordinates u_a.
// ---------------------------------------------------------------------------
// PC: the spline order at compile time (every loop unrolls, the arrays stay in
// registers) or 0 for the order p_rt at run time.
template <int PC>
__device__ inline void mesh_self_term(const double* u, int p_rt, const double* __restrict__ tab, double* val,
                                      double* grad) {
    constexpr int PM = PC ? PC : QEQ_MAXP;
    constexpr int NPM = 2 * PM - 1;
    const int p = PC ? PC : p_rt;
    const int np = 2 * p - 1;
    double R[3][NPM], dR[3][NPM];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double w = u[a] - floor(u[a]);
        double c[QEQ_MAXP], dc[QEQ_MAXP];
        bspline_weights<double>(w, p, c, dc);
#pragma unroll
        for (int d = 0; d < NPM; ++d) {
            R[a][d] = 0.0;
            dR[a][d] = 0.0;
        }
#pragma unroll
        for (int k1 = 0; k1 < PM; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < PM; ++k2) {
                if (!PC && (k1 >= p || k2 >= p)) continue;
                const int d = k2 - k1 + (p - 1);
                R[a][d] += c[k1] * c[k2];
                dR[a][d] += dc[k1] * c[k2] + c[k1] * dc[k2];
            }
    }
    double s = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
    for (int a = 0; a < NPM; ++a)
#pragma unroll
        for (int b = 0; b < NPM; ++b) {
            if (!PC && (a >= np || b >= np)) continue;
            double t = 0.0, t1 = 0.0;
            const double* row = tab + (a * np + b) * np;
#pragma unroll
            for (int c = 0; c < NPM; ++c) {
                if (!PC && c >= np) continue;
                t += row[c] * R[2][c];
                t1 += row[c] * dR[2][c];
            }
            s += R[0][a] * R[1][b] * t;
            g0 += dR[0][a] * R[1][b] * t;
            g1 += R[0][a] * dR[1][b] * t;
            g2 += R[0][a] * R[1][b] * t1;
        }
    *val = s;
    grad[0] = g0;
    grad[1] = g1;
    grad[2] = g2;
}

__device__ __forceinline__ int wrap_idx(int i, int K) {
    i %= K;
    return i < 0 ? i + K : i;
}
