// Host side of the library: plans (device workspace, FFT tables, cell cache),
// the solve / matvec orchestration on the plan's stream, and the C ABI.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "internal.h"

int qeq_check(hipError_t e) {
    if (e == hipSuccess) return QEQ_OK;
    if (e == hipErrorOutOfMemory) return QEQ_ENOMEM;
    return QEQ_EHIP;
}

// ---------------------------------------------------------------- stage timers
static hipEvent_t prof_event(qeq_plan* pl) {
    if (!pl->prof_pool.empty()) {
        hipEvent_t e = pl->prof_pool.back();
        pl->prof_pool.pop_back();
        return e;
    }
    // no system-scope cache fence at the records: the interval is the kernel's
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(qeq_plan* p, int kind) : pl(p) {
    on = kind >= 0 && kind < PK_COUNT && (p->prof_mask >> kind) & 1u;
    rec.kind = kind;
    rec.it = p->cur_it;
    rec.a = rec.b = nullptr;
    if (!on) return;
    rec.a = prof_event(p);
    rec.b = prof_event(p);
    if (!rec.a || !rec.b) on = false;
}

ProfScope::~ProfScope() {
    if (!on) {
        if (rec.a) pl->prof_pool.push_back(rec.a);
        if (rec.b) pl->prof_pool.push_back(rec.b);
        return;
    }
    pl->prof_pending.push_back(rec);
}

// Accumulate the recorded durations (stream already synchronised).  Launches
// of CG iterations at or beyond the number of live iterations found the done
// flag set and returned at once; they are dropped.
void prof_flush(qeq_plan* pl, int live_iters) {
    for (ProfRec& r : pl->prof_pending) {
        float ms = 0.f;
        bool live = r.it < 0 || r.it < live_iters;
        if (live && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            pl->prof_ms[r.kind] += ms;
            pl->prof_n[r.kind] += 1;
        }
        pl->prof_pool.push_back(r.a);
        pl->prof_pool.push_back(r.b);
    }
    pl->prof_pending.clear();
}

void debug_poison(void* p, size_t bytes) {
    if (p && bytes && getenv("QEQ_POISON_ALLOC") != nullptr) (void)hipMemset(p, 0xff, bytes);
}

namespace {

const double PI = 3.14159265358979323846;

template <typename T>
int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return QEQ_ENOMEM;
    if (poisonable<T>) debug_poison(*p, count * sizeof(T));
    return QEQ_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

bool smooth_235(int n) {
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

// Radix plan: all factors 5 and 3 first, then the power of two as 8s with a
// final 4 or 2.
bool radix_plan(int K, FftAxis* ax) {
    int n = K, ns = 0;
    while (n % 5 == 0) { ax->radix[ns++] = 5; n /= 5; }
    while (n % 3 == 0) { ax->radix[ns++] = 3; n /= 3; }
    while (n % 8 == 0) { ax->radix[ns++] = 8; n /= 8; }
    if (n == 4) { ax->radix[ns++] = 4; n = 1; }
    if (n == 2) { ax->radix[ns++] = 2; n = 1; }
    if (n != 1 || ns > QEQ_FFT_MAXST) return false;
    ax->nst = ns;
    ax->K = K;
    return true;
}

// Cardinal B-spline M_p at the integers 0..p (host, FP64).
void bspline_integer_values(int p, double* out) {
    double c[QEQ_MAXP + 1] = {0}, dc[QEQ_MAXP + 1] = {0};
    // weights at w = 0: c[k] = M_p(k)
    c[0] = 0.0;
    c[1] = 1.0;
    for (int k = 2; k <= QEQ_MAXP; ++k) c[k] = 0.0;
    for (int n = 3; n <= p; ++n) {
        double inv = 1.0 / (n - 1);
        for (int k = n - 1; k >= 1; --k) c[k] = (k * c[k] + (n - k) * c[k - 1]) * inv;
        c[0] = 0.0;
    }
    (void)dc;
    for (int k = 0; k <= p; ++k) out[k] = k < QEQ_MAXP + 1 ? c[k] : 0.0;
}

// |b(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2  (Essmann et al.)
void bspline_moduli(int K, int p, std::vector<float>& out) {
    double M[QEQ_MAXP + 1];
    bspline_integer_values(p, M);
    out.resize(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= p - 2; ++k) {
            double a = 2.0 * PI * (double)m * k / K;
            re += M[k + 1] * cos(a);
            im += M[k + 1] * sin(a);
        }
        double d = re * re + im * im;
        out[m] = d > 1e-30 ? (float)(1.0 / d) : 0.f;
    }
}

void inv3(const double* H, double* Hi, double* det) {
    double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7], i = H[8];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double D = -(b * i - c * h), E = a * i - c * g, F = -(a * h - b * g);
    double G = b * f - c * e, Hh = -(a * f - c * d), I = a * e - b * d;
    *det = a * A + b * B + c * C;
    double r = 1.0 / *det;
    Hi[0] = A * r; Hi[1] = D * r; Hi[2] = G * r;
    Hi[3] = B * r; Hi[4] = E * r; Hi[5] = Hh * r;
    Hi[6] = C * r; Hi[7] = F * r; Hi[8] = I * r;
}

double pair_f(double r, double eta, double zeta) {
    const double s2 = 0.70710678118654752440;
    if (r < 1e-12) return sqrt(2.0 / PI) * (1.0 / eta - 1.0 / zeta);
    return (erf(r * s2 / eta) - erf(r * s2 / zeta)) / r;
}

// C_eta = (4 pi / V) sum_{k != 0} exp(-eta^2 k^2 / 2) / k^2 evaluated with a
// second, wider split zeta: C_eta = C_zeta + sum_n f(|n H|) - 2 pi (zeta^2 - eta^2) / V,
// f(r) = [erf(r/(sqrt2 eta)) - erf(r/(sqrt2 zeta))] / r (Poisson summation of
// the difference kernel), which needs few k vectors and few lattice vectors.
double reciprocal_self_constant(const double* H, const double* Hinv, double vol, double eta) {
    double widths[3], lengths[3];
    for (int a = 0; a < 3; ++a) {
        double n2 = 0.0, l2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            n2 += Hinv[c * 3 + a] * Hinv[c * 3 + a];
            l2 += H[a * 3 + c] * H[a * 3 + c];
        }
        widths[a] = 1.0 / sqrt(n2);
        lengths[a] = sqrt(l2);
    }
    double zeta = std::max(eta, 0.3 * cbrt(vol));
    const double X = 6.5 * sqrt(2.0);
    // k-space with zeta
    double kmax = X / zeta;
    int mm[3];
    for (int a = 0; a < 3; ++a) mm[a] = (int)ceil(kmax * lengths[a] / (2 * PI)) + 1;
    double ks = 0.0;
    for (int m1 = -mm[0]; m1 <= mm[0]; ++m1)
        for (int m2 = -mm[1]; m2 <= mm[1]; ++m2)
            for (int m3 = -mm[2]; m3 <= mm[2]; ++m3) {
                if (!m1 && !m2 && !m3) continue;
                double k[3];
                for (int c = 0; c < 3; ++c)
                    k[c] = 2 * PI * (Hinv[c * 3 + 0] * m1 + Hinv[c * 3 + 1] * m2 + Hinv[c * 3 + 2] * m3);
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                if (k2 > kmax * kmax) continue;
                ks += exp(-0.5 * zeta * zeta * k2) / k2;
            }
    ks *= 4 * PI / vol;
    // real-space lattice sum of the difference kernel
    double rmax = X * zeta;
    int nn[3];
    for (int a = 0; a < 3; ++a) nn[a] = (int)ceil(rmax / widths[a]) + 1;
    double rs = 0.0;
    for (int n1 = -nn[0]; n1 <= nn[0]; ++n1)
        for (int n2 = -nn[1]; n2 <= nn[1]; ++n2)
            for (int n3 = -nn[2]; n3 <= nn[2]; ++n3) {
                double x[3];
                for (int c = 0; c < 3; ++c) x[c] = n1 * H[0 * 3 + c] + n2 * H[1 * 3 + c] + n3 * H[2 * 3 + c];
                double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                if (r > rmax) continue;
                rs += pair_f(r, eta, zeta);
            }
    return ks + rs - 2 * PI * (zeta * zeta - eta * eta) / vol;
}

}  // namespace

// d C_eta / d eps_ab for the strain r -> (1 + eps) r, term by term from the
// zeta split above: each k-space term (4 pi / V) e^{-zeta^2 k^2/2} / k^2
// changes by the factor -delta + 2 (1/k^2 + zeta^2/2) k_a k_b, each lattice
// term f(|x|) by f'(r) x_a x_b / r, and -2 pi (zeta^2 - eta^2) / V by
// +2 pi (zeta^2 - eta^2) / V delta.  Order 00, 11, 22, 01, 02, 12.
void reciprocal_self_strain(const double* H, const double* Hinv, double vol, double eta, double dC[6]) {
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    double widths[3], lengths[3];
    for (int a = 0; a < 3; ++a) {
        double n2 = 0.0, l2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            n2 += Hinv[c * 3 + a] * Hinv[c * 3 + a];
            l2 += H[a * 3 + c] * H[a * 3 + c];
        }
        widths[a] = 1.0 / sqrt(n2);
        lengths[a] = sqrt(l2);
    }
    const double zeta = std::max(eta, 0.3 * cbrt(vol));
    const double X = 6.5 * sqrt(2.0);
    for (int c = 0; c < 6; ++c) dC[c] = 0.0;
    const double kmax = X / zeta;
    int mm[3];
    for (int a = 0; a < 3; ++a) mm[a] = (int)ceil(kmax * lengths[a] / (2 * PI)) + 1;
    for (int m1 = -mm[0]; m1 <= mm[0]; ++m1)
        for (int m2 = -mm[1]; m2 <= mm[1]; ++m2)
            for (int m3 = -mm[2]; m3 <= mm[2]; ++m3) {
                if (!m1 && !m2 && !m3) continue;
                double k[3];
                for (int c = 0; c < 3; ++c)
                    k[c] = 2 * PI * (Hinv[c * 3 + 0] * m1 + Hinv[c * 3 + 1] * m2 + Hinv[c * 3 + 2] * m3);
                const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                if (k2 > kmax * kmax) continue;
                const double e = 4 * PI / vol * exp(-0.5 * zeta * zeta * k2) / k2;
                const double cf = 2.0 * (1.0 / k2 + 0.5 * zeta * zeta);
                for (int c = 0; c < 6; ++c) dC[c] += e * ((c < 3 ? -1.0 : 0.0) + cf * k[ia[c]] * k[ib[c]]);
            }
    const double rmax = X * zeta;
    const double a = 0.70710678118654752440 / eta, b = 0.70710678118654752440 / zeta;
    int nn[3];
    for (int t = 0; t < 3; ++t) nn[t] = (int)ceil(rmax / widths[t]) + 1;
    for (int n1 = -nn[0]; n1 <= nn[0]; ++n1)
        for (int n2 = -nn[1]; n2 <= nn[1]; ++n2)
            for (int n3 = -nn[2]; n3 <= nn[2]; ++n3) {
                if (!n1 && !n2 && !n3) continue;
                double x[3];
                for (int c = 0; c < 3; ++c) x[c] = n1 * H[0 * 3 + c] + n2 * H[1 * 3 + c] + n3 * H[2 * 3 + c];
                const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                if (r > rmax) continue;
                const double f = (erf(a * r) - erf(b * r)) / r;
                const double fp = (2.0 / sqrt(PI) * (a * exp(-a * a * r * r) - b * exp(-b * b * r * r)) - f) / r;
                for (int c = 0; c < 6; ++c) dC[c] += fp * x[ia[c]] * x[ib[c]] / r;
            }
    for (int c = 0; c < 3; ++c) dC[c] += 2 * PI * (zeta * zeta - eta * eta) / vol;
}

namespace {

void free_grid(qeq_plan* pl) {
    for (int a = 0; a < 3; ++a) {
        dfree(pl->tw[a]);
        dfree(pl->bmod[a]);
    }
    dfree(pl->grid_r);
    dfree(pl->grid_c);
    dfree(pl->bin_count);
    dfree(pl->bin_start);
    dfree(pl->bin_fill);
    pl->K[0] = pl->K[1] = pl->K[2] = 0;
    pl->theta_valid = false;
    pl->strain_valid = false;
}

int ensure_grid(qeq_plan* pl, const int K[3]) {
    if (pl->K[0] == K[0] && pl->K[1] == K[1] && pl->K[2] == K[2]) return QEQ_OK;
    free_grid(pl);
    int p = pl->prm.spline_order;
    for (int a = 0; a < 3; ++a) {
        if (K[a] < 12 || K[a] > 512 || K[a] % 4 != 0 || !smooth_235(K[a]) || K[a] < 2 * p)
            return QEQ_EPLAN;
    }
    for (int a = 0; a < 3; ++a) {
        FftAxis ax;
        if (!radix_plan(K[a], &ax)) return QEQ_EPLAN;
        std::vector<float2> tw(K[a]);
        for (int j = 0; j < K[a]; ++j) {
            double ang = -2.0 * PI * (double)j / (double)K[a];
            tw[j] = make_float2((float)cos(ang), (float)sin(ang));
        }
        QEQ_TRY(dalloc(&pl->tw[a], K[a]));
        QEQ_HIP(hipMemcpy(pl->tw[a], tw.data(), sizeof(float2) * K[a], hipMemcpyHostToDevice));
        ax.tw = pl->tw[a];
        pl->axes.ax[a] = ax;
        std::vector<float> bm;
        bspline_moduli(K[a], p, bm);
        QEQ_TRY(dalloc(&pl->bmod[a], K[a]));
        QEQ_HIP(hipMemcpy(pl->bmod[a], bm.data(), sizeof(float) * K[a], hipMemcpyHostToDevice));
    }
    size_t nreal = (size_t)K[0] * K[1] * K[2];
    size_t ncplx = (size_t)(K[2] / 2 + 1) * K[0] * K[1];
    QEQ_TRY(dalloc(&pl->grid_r, nreal));
    QEQ_TRY(dalloc(&pl->grid_c, ncplx));
    int nb = K[0] * K[1] + 1;
    QEQ_TRY(dalloc(&pl->bin_count, nb));
    QEQ_TRY(dalloc(&pl->bin_start, nb + 1));
    QEQ_TRY(dalloc(&pl->bin_fill, nb));
    pl->grid_bytes = nreal * 4 + ncplx * 8;
    pl->K[0] = K[0];
    pl->K[1] = K[1];
    pl->K[2] = K[2];
    pl->theta_valid = false;
    pl->strain_valid = false;
    return QEQ_OK;
}

int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Geometry, grid and kernel parameters for one call.
int prepare(qeq_plan* pl, int n, const double* cell, double q_tot) {
    if (n < 1 || !cell) return QEQ_EINVAL;
    if (n > pl->n_max) return QEQ_EPLAN;
    for (int t = 0; t < 9; ++t)
        if (!isfinite(cell[t])) return QEQ_EINVAL;
    if (!isfinite(q_tot)) return QEQ_EINVAL;
    KParams& k = pl->kp;
    memset(&k, 0, sizeof(k));
    double det;
    double Hi[9];
    inv3(cell, Hi, &det);
    if (!(det > 0.0) || !isfinite(det)) return QEQ_EINVAL;
    for (int t = 0; t < 9; ++t) {
        k.H[t] = cell[t];
        k.Hinv[t] = Hi[t];
    }
    k.vol = det;
    // metric (H H^T)^-1 = Hinv^T Hinv
    double Mm[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Hi[c * 3 + a] * Hi[c * 3 + b];
            Mm[a * 3 + b] = s;
        }
    k.M[0] = Mm[0];
    k.M[1] = Mm[4];
    k.M[2] = Mm[8];
    k.M[3] = Mm[1];
    k.M[4] = Mm[2];
    k.M[5] = Mm[5];
    double widths[3], lengths[3];
    for (int a = 0; a < 3; ++a) {
        widths[a] = 1.0 / sqrt(Mm[a * 3 + a]);
        lengths[a] = sqrt(cell[a * 3] * cell[a * 3] + cell[a * 3 + 1] * cell[a * 3 + 1] +
                          cell[a * 3 + 2] * cell[a * 3 + 2]);
    }
    int K[3];
    for (int a = 0; a < 3; ++a) {
        if (pl->prm.grid[0] > 0) {
            K[a] = pl->prm.grid[a];
        } else {
            int m = (int)ceil(lengths[a] / pl->prm.max_spacing - 1e-12);
            m = std::max(m, 12);
            m = (m + 3) / 4 * 4;
            while (!smooth_235(m)) m += 4;
            K[a] = m;
        }
    }
    QEQ_TRY(ensure_grid(pl, K));
    const int p = pl->prm.spline_order;
    k.n = n;
    k.p = p;
    k.K1 = K[0];
    k.K2 = K[1];
    k.K3 = K[2];
    k.K3h = K[2] / 2 + 1;
    // Axis-1 / complex-to-real tiles of 16, 8 or 4 rows, every pass's block
    // within 48 KB of LDS.  16 rows at 192^3 and at 320^3: with the
    // two-stage transforms a 16-column tile keeps every thread of a radix-20
    // stage busy (320^3: axis-1 pass 66.3 -> 49.9 us, C2R 49.7 -> 45.4 us
    // against 8 rows); 32 rows were slower everywhere.
    auto tile_fits = [&](int t) {
        return K[1] % t == 0 && (size_t)K[0] * t * 8 <= 49152 &&
               (size_t)K[2] * (t / 2) * 8 + (size_t)(K[2] / 2 + 1) * t * 8 <= 49152;
    };
    // Spread tiles (block LDS: twiddles + int32 accumulator of the tile):
    // the widest compiled width whose block stays within 26 KB (six blocks
    // fit a CU) and that still gives at least two blocks per CU; failing
    // that the widest compiled one within 26 KB; failing that the runtime
    // kernel's power-of-two widths within 32 KB.  The spread's blocks wait
    // mostly on their own chain of loads, atomics and barriers, so few,
    // wide tiles that start together beat many narrow ones: 192^3, 24 rows
    // (1,536 blocks, one round): 17.6 us per launch against 19.1 for 12
    // rows; 320^3, 16 rows: 52.9 us against 55.7 for 8.
    auto spread_fits = [&](int w) {
        return K[1] % w == 0 && K[1] >= w + p - 1 && spread_tile_compiled(K[2], w, p) &&
               (size_t)K[2] * 8 + (size_t)K[2] * w * 4 <= 26624;
    };
    int tws = 0;
    for (int w : {32, 24, 16, 12, 8})
        if (!tws && spread_fits(w) && (size_t)K[0] * (K[1] / w) >= 512) tws = w;
    for (int w : {32, 24, 16, 12, 8})
        if (!tws && spread_fits(w)) tws = w;
    if (!tws) {
        tws = 16;
        while (tws > 4 && (K[1] % tws != 0 || (size_t)K[2] * 8 + (size_t)K[2] * tws * 4 > 32768)) tws >>= 1;
    }
    int tw = 16;
    while (tw > 4 && !tile_fits(tw)) tw >>= 1;
    // tile widths set with qeq_set_tiles (e.g. by the autotuner) replace the rule
    if (pl->tile_set[0] > 0) tws = pl->tile_set[0];
    if (pl->tile_set[1] > 0) tw = pl->tile_set[1];
    if (K[1] % tws != 0 || K[1] < tws + p - 1) return QEQ_EPLAN;
    if (K[1] % tw != 0 || K[1] < tw + p - 1) return QEQ_EPLAN;
    if ((size_t)K[2] * 8 + (size_t)K[2] * tws * 4 > 61440 || (size_t)K[0] * tw * 8 + K[0] * 8 > 61440 ||
        (size_t)K[2] * (tw / 2) * 8 + (size_t)(K[2] / 2 + 1) * tw * 8 + K[2] * 8 > 61440)
        return QEQ_EPLAN;
    k.TW = tw;
    k.TWlog2 = ilog2(tw);
    k.ntile = K[1] / tw;
    k.TWS = tws;
    k.ntile_s = K[1] / tws;
    int nr = 16;
    while (nr > 1 && (size_t)K[1] * nr * 8 > 32768) nr >>= 1;
    // grids beyond the ~256 MB Infinity Cache stream from HBM: there 4 rows
    // per block of the axis-2 pass overlap better (320^3: 58 / 54 -> 53 /
    // 46 us); cache-resident grids keep the larger blocks
    const size_t grid_bytes = (size_t)K[0] * K[1] * K[2] * 4 + (size_t)K[0] * K[1] * (K[2] / 2 + 1) * 8;
    if (grid_bytes > ((size_t)192 << 20) && nr > 4) nr = 4;
    if (pl->tile_set[2] > 0) nr = pl->tile_set[2];
    if ((size_t)K[1] * (nr + 2) * 8 > 61440) return QEQ_EPLAN;
    k.NR = nr;
    k.NRlog2 = ilog2(nr);
    // every FFT stage must fit the per-thread register budget
    if ((size_t)K[0] * tw > (size_t)QEQ_FFT_EMAX * QEQ_FFT_THREADS ||
        (size_t)K[1] * nr > (size_t)QEQ_FFT_EMAX * QEQ_FFT_THREADS ||
        (size_t)K[2] * (tw / 2) > (size_t)QEQ_FFT_EMAX * QEQ_FFT_THREADS)
        return QEQ_EPLAN;
    // real-space cells: at least half a cutoff wide
    double rc = pl->prm.r_cut;
    int ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int nc = (int)floor(2.0 * widths[a] / rc);
        nc = std::max(1, std::min(nc, 256));
        k.nc[a] = nc;
        k.ns[a] = (int)ceil(rc * nc / widths[a] - 1e-12);
        if (k.ns[a] > 64) return QEQ_ECELL;
        ncell *= nc;
    }
    if (ncell + 1 > pl->ncell_alloc) {
        dfree(pl->cell_count);
        dfree(pl->cell_start);
        dfree(pl->cell_fill);
        QEQ_TRY(dalloc(&pl->cell_count, ncell + 1));
        QEQ_TRY(dalloc(&pl->cell_start, ncell + 2));
        QEQ_TRY(dalloc(&pl->cell_fill, ncell + 1));
        pl->ncell_alloc = ncell + 1;
    }
    // with direct Ewald sums the reciprocal part is added from outside the
    // interpolation pass and is exact (no mesh self-correction)
    // The Gaussian-on-grid operator is the whole Coulomb operator of the
    // periodic densities (no split: no real-space pairs, no self or
    // background terms, no screening in the Green's function).
    const bool ext_rec = pl->ew_active || pl->pw_active;
    k.parts = (ext_rec ? 0 : QEQ_PART_RECIP) |
              (pl->pw_active ? 0 : (QEQ_PART_REAL | QEQ_PART_SELF | QEQ_PART_BG));
    k.self_corr = ext_rec ? 0 : pl->prm.self_correction;
    k.eta = pl->prm.eta;
    k.eta_green = pl->pw_active ? 0.0 : pl->prm.eta;
    k.rc = rc;
    k.rc2 = rc * rc;
    k.green_pref = 4.0 * PI / det;
    k.bg_pref = pl->pw_active ? 0.0 : 2.0 * PI / det;
    k.q_tot = q_tot;
    k.tol = pl->prm.tol;
    bool same_cell = true;
    for (int t = 0; t < 9; ++t) same_cell = same_cell && (pl->cell_cached[t] == cell[t]);
    if (!same_cell || !pl->theta_valid) {
        pl->c_eta = reciprocal_self_constant(k.H, k.Hinv, det, k.eta);
        pl->theta_valid = false;
        pl->strain_valid = false;
    }
    k.c_eta = pl->c_eta;
    if (k.self_corr && !pl->theta_valid) {
        QEQ_TRY(launch_theta(pl));
        pl->theta_valid = true;
    }
    for (int t = 0; t < 9; ++t) pl->cell_cached[t] = cell[t];
    return QEQ_OK;
}

// Geometry-dependent setup on the device; one host sync (pair count, input flag).
int setup_geometry(qeq_plan* pl, const double* pos, const double* sigma, const double* J,
                   const double* chi) {
    QEQ_TRY(launch_setup_clear(pl));   // CG scalars, bin and cell counters
    QEQ_TRY(launch_stage(pl, pos, sigma, J, chi));
    QEQ_TRY(launch_sort_bins(pl));
    QEQ_TRY(launch_gather(pl, pos, sigma, J, chi));
    QEQ_TRY(launch_cells_and_pairs(pl));
    // one read-back for the input check and the pair count
    QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    if (pl->sc_host->err & QEQ_ERRBIT_INPUT) return QEQ_EINVAL;
    pl->nnz = *pl->nnz_host;
    if ((size_t)pl->nnz > pl->nnz_cap) {   // rows past the capacity were skipped: grow and fill again
        QEQ_TRY(grow_pairs(pl, (size_t)(pl->nnz * 1.25) + 1024));
        QEQ_TRY(launch_pair_fill(pl));
    }
    if (pl->kp.self_corr) QEQ_TRY(launch_selfcorr(pl));
    return QEQ_OK;
}

// Bytes that determine the kernels of one CG chunk: the kernel-argument
// bundle and every buffer the chunk touches.
void chunk_key(const qeq_plan* pl, std::vector<unsigned char>& key) {

    const void* ptrs[] = {pl->pvec, pl->y, pl->q, pl->r, pl->dinv, pl->part, pl->sc, pl->grid_r, pl->grid_c,
                          pl->wts, pl->dwts, pl->home, pl->bin_start, pl->rowptr, pl->col, pl->kval, pl->pdr,
                          pl->dself, pl->Jv, pl->chi_raw, pl->chi, pl->sig, pl->selfgrad, pl->fdst, pl->gtmp,
                          pl->tw[0], pl->tw[1], pl->tw[2], pl->bmod[0], pl->bmod[1], pl->bmod[2],
                          pl->spc_active ? (const void*)pl->spc_mats : nullptr, pl->spc_wvec, pl->spc_m1,
                          pl->spc_atom, pl->spc_dpinv, pl->spc_tpart, pl->spc_s, pl->spc_scal,
                          pl->spc_sd, pl->spc_u, pl->spc_psi, (const void*)(size_t)pl->spc_nm,
                          (const void*)(size_t)pl->spc_npad, (const void*)(size_t)pl->direct, pl->np_pos,
                          pl->np_ypart, (const void*)(size_t)pl->np_nsplit, (const void*)(size_t)pl->np_tps,
                          (const void*)(size_t)pl->ew_active, pl->ew_modes, pl->ew_w, pl->ew_sf, pl->ew_y,
                          pl->ew_yrec, (const void*)(size_t)pl->ew_nm, (const void*)(size_t)pl->ew_fs,
                          (const void*)(size_t)pl->ew_ms, (const void*)(size_t)pl->pw_active, pl->pw_ones,
                          pl->pw_y, pl->pw_f};
    key.resize(sizeof(KParams) + sizeof(ptrs) + sizeof(DeviceAxes) + sizeof(PwGeom));
    unsigned char* k = key.data();
    memcpy(k, &pl->kp, sizeof(KParams));
    memcpy(k + sizeof(KParams), ptrs, sizeof(ptrs));
    memcpy(k + sizeof(KParams) + sizeof(ptrs), &pl->axes, sizeof(DeviceAxes));
    memcpy(k + sizeof(KParams) + sizeof(ptrs) + sizeof(DeviceAxes), &pl->pw_geom, sizeof(PwGeom));
}

void drop_graph(qeq_plan* pl) {
    if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->graph_exec = nullptr;
    pl->graph = nullptr;
    pl->graph_key.clear();
}

// One CG iteration: matvec of the direction, update of q and r, new direction.
// Search direction from the current residual: Jacobi, or the spectral
// preconditioner when it was built for this geometry.
// u_ready: the update kernel has already written the spectral
// preconditioner's input from r.
int next_direction(qeq_plan* pl, int parity, int init, bool u_ready = false) {
    if (!pl->spc_active) return launch_cg_dir(pl, parity, init);
    QEQ_TRY(spc_apply(pl, pl->r, &pl->sc->done, u_ready));
    return spc_direction(pl, parity, init);
}

// y = A src with the CG partial sums: the particle-mesh operator, or the
// direct pair sum of an isolated system.
int cg_matvec(qeq_plan* pl, const double* src, int parity) {
    if (pl->direct) return launch_np_matvec(pl, src, pl->y, QEQ_MODE_CG);
    if (pl->ew_active) {
        QEQ_TRY(launch_ew_rec(pl, src, &pl->sc->done, false));
        return launch_interp(pl, src, pl->y, QEQ_MODE_CG, parity);
    }
    if (pl->pw_active) {
        QEQ_TRY(launch_pw_rec(pl, src, &pl->sc->done, false));
        return launch_interp(pl, src, pl->y, QEQ_MODE_CG, parity);
    }
    bool partials = false;
    QEQ_TRY(launch_mesh_cg(pl, src, &pl->sc->done, &partials));
    return launch_interp(pl, src, pl->y, QEQ_MODE_CG, parity, partials ? pl->mpart : nullptr);
}

int cg_iteration(qeq_plan* pl, int parity) {
    QEQ_TRY(cg_matvec(pl, pl->pvec, parity));
    QEQ_TRY(launch_cg_update(pl, parity));
    return next_direction(pl, parity, 0, true);
}

// Capture `chunk` iterations (starting at even parity) into a graph unless the
// current one was captured with the same arguments.  Every kernel of the loop
// reads the device flag `done` and returns at once after convergence, so the
// graph can be replayed whole.
int ensure_chunk_graph(qeq_plan* pl, int chunk) {
    std::vector<unsigned char> key;
    chunk_key(pl, key);
    // the captured length is part of the key
    const unsigned char* cb = reinterpret_cast<const unsigned char*>(&chunk);
    key.insert(key.end(), cb, cb + sizeof(chunk));
    if (pl->graph_exec && key == pl->graph_key) return QEQ_OK;
    drop_graph(pl);
    if (!pl->cap_stream) QEQ_HIP(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    hipStream_t user = pl->stream;
    pl->stream = pl->cap_stream;
    int rc = qeq_check(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    if (rc == QEQ_OK) {
        for (int t = 0; t < chunk && rc == QEQ_OK; ++t) rc = cg_iteration(pl, t & 1);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
        if (rc == QEQ_OK) rc = qeq_check(e);
        if (rc == QEQ_OK) {
            rc = qeq_check(hipGraphInstantiate(&pl->graph_exec, g, nullptr, nullptr, 0));
            pl->graph = g;
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    pl->stream = user;
    if (rc != QEQ_OK) {
        drop_graph(pl);
        return rc;
    }
    pl->graph_key.swap(key);
    return QEQ_OK;
}


}  // namespace

// Final product on q: energies, mu, true residual, forces; scatter to caller
// order; host copies of the results and of the CG scalars.
int final_pass(qeq_plan* pl, double* q_out, double* energies, double* forces_out) {
    if (pl->direct) {
        QEQ_TRY(launch_np_matvec(pl, pl->q, pl->y, QEQ_MODE_FINAL));
        QEQ_TRY(launch_final_tail(pl, q_out, energies, forces_out));
    } else if (pl->ew_active) {
        QEQ_TRY(launch_ew_rec(pl, pl->q, nullptr, true));
        QEQ_TRY(launch_final(pl, q_out, energies, forces_out));
    } else if (pl->pw_active) {
        QEQ_TRY(launch_pw_rec(pl, pl->q, nullptr, true));
        QEQ_TRY(launch_final(pl, q_out, energies, forces_out));
    } else {
        QEQ_TRY(launch_mesh_potential(pl, pl->q, nullptr));
        QEQ_TRY(launch_final(pl, q_out, energies, forces_out));
    }
    QEQ_HIP(hipMemcpyAsync(pl->out_host, pl->final_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    return QEQ_OK;
}

// dst = E src (sorted order, no J, no partial sums) with the solve's operator.
int operator_product(qeq_plan* pl, const double* src, double* dst) {
    if (pl->ew_active) {
        QEQ_TRY(launch_ew_rec(pl, src, nullptr, false));
    } else if (pl->pw_active) {
        QEQ_TRY(launch_pw_rec(pl, src, nullptr, false));
    } else {
        QEQ_TRY(launch_mesh_potential(pl, src, nullptr));
    }
    return launch_interp(pl, src, dst, QEQ_MODE_MATVEC, 0);
}

namespace {

// Projected CG from q0 (or Q/N) to the tolerance, with the true-residual
// restart, then the final matvec: energies, mu, true residual and forces are
// computed; q_out / energies / forces_out (caller order) may be NULL.
int cg_run(qeq_plan* pl, const double* q0, double* q_out, double* energies, double* forces_out,
           bool* conv_out) {
    const int* done = &pl->sc->done;
    pl->warm_rejected = false;
    // initial guess (projected onto the constraint plane)
    QEQ_TRY(launch_cg_init_q(pl, q0));
    // iterations per replayed graph: 12 for the Jacobi solves (57-125
    // iterations here), 4 with the spectral preconditioner (17-29), whose
    // early-returning launches after convergence would outweigh the saved
    // graph launches of longer chunks
    const int chunk = pl->spc_active ? 4 : 12;
    int it = 0;
    bool conv = false;
    // The recursive residual of CG drifts from the true one by the FP32 error
    // of the matvecs, which scales with |q| along the way.  After convergence
    // the final matvec (which also yields energies and forces) measures the
    // true residual; above 2 max(tol, 1e-7) CG restarts from the current
    // charges (at most four times).  A solve that still ends above it is
    // reported converged if the true residual is within twice the FP32 floor
    // of the products: ~2e-7 at 32,768 atoms, 2.3e-7 to 4.1e-7 (median
    // 3.3e-7) after the restarts in cold solves of 131,072-atom trajectory
    // frames at tol 2e-7, so 2 max(tol, 3e-7).
    const double restart_thr = 2.0 * std::max(pl->prm.tol, 1e-7);
    const double accept_thr = 2.0 * std::max(pl->prm.tol, 3e-7);
    for (int restart = 0;; ++restart) {
        // residual of the current q and the first direction
        QEQ_TRY(cg_matvec(pl, pl->q, 0));
        QEQ_TRY(launch_cg_init_r(pl));
        QEQ_TRY(next_direction(pl, 1, 1));
        if (restart == 0 && q0) {
            // A supplied guess is kept only if it starts closer to the solution
            // than the cold start in the energy norm that CG minimises: for
            // Q_tot = 0 the cold start q = 0 has energy 0, so a guess with
            // E(q0) = 1/2 q0.A q0 + chi_eff.q0 >= 0 is replaced; for charged
            // cells the relative residual (1 for the cold start) decides.
            QEQ_TRY(launch_start_energy(pl));
            QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
            QEQ_HIP(hipStreamSynchronize(pl->stream));
            const bool worse = pl->kp.q_tot == 0.0 ? !(pl->sc_host->e_start < 0.0) : !(pl->sc_host->res <= 1.0);
            if (worse) {
                pl->warm_rejected = true;
                QEQ_TRY(launch_cg_init_q(pl, nullptr));
                QEQ_TRY(cg_matvec(pl, pl->q, 0));
                QEQ_TRY(launch_cg_init_r(pl));
                QEQ_TRY(next_direction(pl, 1, 1));
            }
        }
        conv = false;
        int local = 0;
        // Each chunk's scalars are copied to a pinned ring slot behind it.
        // While the last residual seen is far above the tolerance (more than
        // two chunks of CG reduction away), the next chunk is launched before
        // the host waits for the copy, so the GPU does not idle during the
        // read-back; near convergence the host waits after every chunk, so
        // at most one chunk of early-returning kernels is ever launched in
        // vain.
        if (!pl->ring_ev[0]) {
            for (int e = 0; e < 2; ++e)
                QEQ_HIP(hipEventCreateWithFlags(&pl->ring_ev[e], hipEventDisableTiming));
        }
        int slot = 0, prev = -1;
        double res_seen = 1e300;
        const double ahead_thr = 20.0 * pl->prm.tol;
        bool stop = false;
        while (it < pl->prm.max_iter && !stop) {
            int m = std::min(chunk, pl->prm.max_iter - it);
            // per-stage timers need eager launches (events recorded inside a
            // graph cannot be read back with hipEventElapsedTime)
            if (m == chunk && (local & 1) == 0 && pl->use_graphs && pl->prof_mask == 0) {
                QEQ_TRY(ensure_chunk_graph(pl, chunk));
                QEQ_HIP(hipGraphLaunch(pl->graph_exec, pl->stream));
                it += m;
                local += m;
            } else {
                for (int t = 0; t < m; ++t, ++it, ++local) {
                    pl->cur_it = it;
                    QEQ_TRY(cg_iteration(pl, local & 1));
                }
            }
            pl->cur_it = -1;
            QEQ_HIP(hipMemcpyAsync(&pl->sc_ring[slot], pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost,
                                   pl->stream));
            QEQ_HIP(hipEventRecord(pl->ring_ev[slot], pl->stream));
            if (prev >= 0) {   // the chunk before this one
                QEQ_HIP(hipEventSynchronize(pl->ring_ev[prev]));
                if (pl->sc_ring[prev].done) break;
                res_seen = pl->sc_ring[prev].res;
                prev = -1;
            }
            if (res_seen > ahead_thr && pl->prof_mask == 0) {
                prev = slot;   // go on without waiting for this chunk
            } else {
                QEQ_HIP(hipEventSynchronize(pl->ring_ev[slot]));
                stop = pl->sc_ring[slot].done != 0;
                res_seen = pl->sc_ring[slot].res;
            }
            slot ^= 1;
        }
        QEQ_HIP(hipMemcpyAsync(pl->sc_host, pl->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, pl->stream));
        QEQ_HIP(hipStreamSynchronize(pl->stream));
        conv = pl->sc_host->done != 0;
        QEQ_TRY(final_pass(pl, q_out, energies, forces_out));
        bool gap = !(pl->out_host[3] <= restart_thr);
        if (!conv || !gap || restart >= 4 || it >= pl->prm.max_iter) {
            if (conv && gap) conv = pl->out_host[3] <= accept_thr;
            break;
        }
        QEQ_HIP(hipMemsetAsync(&pl->sc->done, 0, sizeof(int), pl->stream));
    }
    prof_flush(pl, pl->sc_host->iters);
    *conv_out = conv;
    return QEQ_OK;
}

int cg_status(qeq_plan* pl, bool conv, qeq_stats* stats) {
    int status = conv ? QEQ_OK : QEQ_NOT_CONVERGED;
    if (pl->sc_host->err & QEQ_ERRBIT_INPUT) status = QEQ_EINVAL;
    if (!isfinite(pl->out_host[0])) status = status == QEQ_OK ? QEQ_NOT_CONVERGED : status;
    if (stats) {
        stats->status = status;
        stats->iters = pl->sc_host->iters;
        stats->rel_resid = pl->sc_host->res;
        stats->true_rel_resid = pl->out_host[3];
        stats->mu = pl->out_host[2];
        stats->e_qeq = pl->out_host[0];
        stats->e_elec = pl->out_host[1];
        stats->q0_rejected = pl->warm_rejected ? 1 : 0;
        stats->reserved = 0;
    }
    return status;
}

int solve_impl(qeq_plan* pl, int n, const double* pos, const double* cell, const double* sigma,
               const double* J, const double* chi, double q_tot, const double* q0, double* q,
               double* energies, double* forces, qeq_stats* stats) {
    if (!pos || !sigma || !J || !chi || !q) return QEQ_EINVAL;
    pl->tape_valid = false;
    pl->direct = false;
    pl->np_valid = false;
    pl->geom_valid = false;
    pl->ew_active = pl->ewald;
    pl->pw_active = pl->planewave;
    QEQ_TRY(prepare(pl, n, cell, q_tot));
    QEQ_TRY(setup_geometry(pl, pos, sigma, J, chi));
    pl->geom_valid = true;
    if (pl->ew_active) QEQ_TRY(ew_setup(pl));
    if (pl->pw_active) QEQ_TRY(pw_setup(pl));
    QEQ_TRY(spc_setup(pl));
    pl->fdst = pl->forces_s;
    bool conv = false;
    if (pl->sqnm)
        QEQ_TRY(sqnm_run(pl, q0, q, energies, forces, &conv));
    else
        QEQ_TRY(cg_run(pl, q0, q, energies, forces, &conv));
    int status = cg_status(pl, conv, stats);
    // the adjoint, the virial and the element potentials use the split
    // mesh operator: they follow its solves only
    pl->tape_valid = status >= 0 && !pl->ew_active && !pl->pw_active;
    return status;
}

// Adjoint of the solve (SI eq. 4g_force_trick, Lagrange route): one more
// projected CG with the same operator and right-hand side g, then the
// bilinear position derivative of a^T E q from two mesh potentials.
int backward_impl(qeq_plan* pl, const double* dL_dq, double dL_dEelec, double dL_dEqeq, double* dL_dchi,
                  double* dL_dJ, double* dL_dpos, qeq_stats* stats) {
    if (!pl->tape_valid) return QEQ_EINVAL;
    if (!isfinite(dL_dEqeq) || !isfinite(dL_dEelec)) return QEQ_EINVAL;
    const double q_tot = pl->kp.q_tot;
    QEQ_TRY(launch_adj_rhs(pl, dL_dq, dL_dEelec));
    // the adjoint system: A a + nu 1 = g, sum(a) = 0
    // y (= E q of the solve) is part of the tape: the adjoint CG works on a copy
    std::swap(pl->q, pl->q_adj);
    std::swap(pl->chi, pl->chi_adj);
    std::swap(pl->y, pl->y_adj);
    pl->kp.q_tot = 0.0;
    pl->fdst = pl->adj_scratch;
    bool conv = false;
    int rc = cg_run(pl, nullptr, nullptr, nullptr, nullptr, &conv);
    std::swap(pl->q, pl->q_adj);
    std::swap(pl->chi, pl->chi_adj);
    std::swap(pl->y, pl->y_adj);
    pl->kp.q_tot = q_tot;
    pl->fdst = pl->forces_s;
    QEQ_TRY(rc);
    int status = cg_status(pl, conv, stats);
    if (status < 0) return status;
    QEQ_TRY(launch_adj_gradients(pl, dL_dEqeq, dL_dEelec, dL_dchi, dL_dJ, dL_dpos));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    return status;
}

}  // namespace

extern "C" {

void qeq_params_default(qeq_params* p) {
    if (!p) return;
    p->eta = 2.0;
    p->r_cut = 11.0;
    p->max_spacing = 0.8;
    p->grid[0] = p->grid[1] = p->grid[2] = 0;
    p->spline_order = 6;
    p->tol = 1e-6;
    p->max_iter = 1000;
    p->self_correction = 1;
    p->precond = 0;
    p->spectral_kcut = 0.2;
}

int qeq_plan_create(qeq_plan** out, const qeq_params* params, int32_t n_atoms_max, void* hip_stream) {
    if (!out || !params || n_atoms_max < 1) return QEQ_EINVAL;
    *out = nullptr;
    const qeq_params& p = *params;
    if (!(p.eta > 0.0) || !(p.r_cut > 0.0) || !(p.tol > 0.0) || p.max_iter < 0) return QEQ_EINVAL;
    if (p.grid[0] <= 0 && !(p.max_spacing > 0.0)) return QEQ_EINVAL;
    if (p.spline_order < 4 || p.spline_order > QEQ_MAXP || (p.spline_order & 1)) return QEQ_EPLAN;
    if (p.precond != 0 && p.precond != 1) return QEQ_EINVAL;
    if (!(p.spectral_kcut == p.spectral_kcut)) return QEQ_EINVAL;
    qeq_plan* pl = new (std::nothrow) qeq_plan();
    if (!pl) return QEQ_ENOMEM;
    pl->prm = p;
    pl->n_max = n_atoms_max;
    pl->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&pl->dev);
    size_t n = (size_t)n_atoms_max;
    int rc = QEQ_OK;
    auto A = [&](int r) {
        if (rc == QEQ_OK) rc = r;
    };
    A(dalloc(&pl->perm, n));
    A(dalloc(&pl->key, n));
    A(dalloc(&pl->frac, 3 * n));
    A(dalloc(&pl->home, 4 * n));
    A(dalloc(&pl->wts, 3 * QEQ_MAXP * n));
    A(dalloc(&pl->dwts, 3 * QEQ_MAXP * n));
    A(dalloc(&pl->sig, n));
    A(dalloc(&pl->Jv, n));
    A(dalloc(&pl->chi, n));
    A(dalloc(&pl->chi_raw, n));
    A(dalloc(&pl->dself, n));
    A(dalloc(&pl->dinv, n));
    A(dalloc(&pl->selfgrad, 3 * n));
    A(dalloc(&pl->q, n));
    A(dalloc(&pl->r, n));
    A(dalloc(&pl->pvec, n));
    A(dalloc(&pl->y, n));
    A(dalloc(&pl->forces_s, 3 * n));
    A(dalloc(&pl->gtmp, n));
    A(dalloc(&pl->q_adj, n));
    A(dalloc(&pl->y_adj, n));
    A(dalloc(&pl->chi_adj, n));
    A(dalloc(&pl->adj_scratch, 3 * n));
    A(dalloc(&pl->tq, 3 * n));
    A(dalloc(&pl->mpart, 2 * QEQ_MAXP * n));
    pl->fdst = pl->forces_s;
    A(dalloc(&pl->rowptr, n + 1));
    A(dalloc(&pl->cell_atoms, n));
    A(dalloc(&pl->rowcnt, n + 1));
    A(dalloc(&pl->lanecnt, (size_t)64 * n));
    int np = 2 * QEQ_MAXP - 1;
    A(dalloc(&pl->theta_tab, (size_t)np * np * np));
    pl->nblk_max = std::max(interp_blocks(n_atoms_max), nblocks(n_atoms_max)) + 1;   // most blocks of any reduction
    A(dalloc(&pl->part, (size_t)2 * pl->nblk_max * QEQ_NPART));
    A(dalloc(&pl->sc, 1));
    A(dalloc(&pl->final_dev, 16));
    if (rc == QEQ_OK && hipHostMalloc((void**)&pl->sc_host, sizeof(CgScalars)) != hipSuccess) rc = QEQ_ENOMEM;
    if (rc == QEQ_OK && hipHostMalloc((void**)&pl->out_host, 16 * sizeof(double)) != hipSuccess)
        rc = QEQ_ENOMEM;
    if (rc == QEQ_OK && hipHostMalloc((void**)&pl->nnz_host, sizeof(int)) != hipSuccess) rc = QEQ_ENOMEM;
    if (rc == QEQ_OK && hipHostMalloc((void**)&pl->sc_ring, 2 * sizeof(CgScalars)) != hipSuccess)
        rc = QEQ_ENOMEM;
    if (rc == QEQ_OK && p.grid[0] > 0) rc = ensure_grid(pl, p.grid);
    if (p.precond == 1) pl->spc_kc = p.spectral_kcut > 0.0 ? p.spectral_kcut : 0.2;
    if (rc != QEQ_OK) {
        qeq_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return QEQ_OK;
}

int qeq_plan_destroy(qeq_plan* pl) {
    if (!pl) return QEQ_OK;
    if (pl->stream) (void)hipStreamSynchronize(pl->stream);
    prof_flush(pl, 0);
    for (hipEvent_t e : pl->prof_pool) (void)hipEventDestroy(e);
    pl->prof_pool.clear();
    drop_graph(pl);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    free_grid(pl);
    batch_free(pl);
    dfree(pl->perm); dfree(pl->key); dfree(pl->frac); dfree(pl->home); dfree(pl->wts); dfree(pl->dwts);
    dfree(pl->sig); dfree(pl->Jv); dfree(pl->chi); dfree(pl->chi_raw); dfree(pl->dself); dfree(pl->dinv);
    dfree(pl->selfgrad); dfree(pl->q); dfree(pl->r); dfree(pl->pvec); dfree(pl->y); dfree(pl->forces_s);
    dfree(pl->gtmp); dfree(pl->q_adj); dfree(pl->y_adj); dfree(pl->chi_adj); dfree(pl->adj_scratch); dfree(pl->tq); dfree(pl->rowptr); dfree(pl->rowcnt); dfree(pl->lanecnt); dfree(pl->theta_tab); dfree(pl->part);
    dfree(pl->strain_tab); dfree(pl->vir_part); dfree(pl->mpart);
    spc_free(pl);
    np_free(pl);
    ew_free(pl);
    pw_free(pl);
    sqnm_free(pl);
    if (pl->elem_buf) (void)hipFree(pl->elem_buf);
    dfree(pl->sc); dfree(pl->final_dev); dfree(pl->scan_tmp);
    dfree(pl->cell_count); dfree(pl->cell_start); dfree(pl->cell_fill); dfree(pl->cell_atoms);
    dfree(pl->col); dfree(pl->kval); dfree(pl->pdr);
    if (pl->sc_host) (void)hipHostFree(pl->sc_host);
    if (pl->out_host) (void)hipHostFree(pl->out_host);
    if (pl->nnz_host) (void)hipHostFree(pl->nnz_host);
    for (int e = 0; e < 2; ++e)
        if (pl->ring_ev[e]) (void)hipEventDestroy(pl->ring_ev[e]);
    if (pl->sc_ring) (void)hipHostFree(pl->sc_ring);
    delete pl;
    return QEQ_OK;
}

int qeq_solve(qeq_plan* plan, int32_t n, const double* pos, const double* cell, const double* sigma,
              const double* J, const double* chi, double q_tot, const double* q0, double* q,
              double* energies, double* forces, qeq_stats* stats) {
    if (!plan) return QEQ_EINVAL;
    int rc = solve_impl(plan, n, pos, cell, sigma, J, chi, q_tot, q0, q, energies, forces, stats);
    if (rc < 0 && stats) {
        memset(stats, 0, sizeof(*stats));
        stats->status = rc;
    }
    return rc;
}

int qeq_solve_nonperiodic(qeq_plan* plan, int32_t n, const double* pos, const double* sigma, const double* J,
                          const double* chi, double q_tot, const double* q0, double* q, double* energies,
                          double* forces, qeq_stats* stats) {
    if (!plan) return QEQ_EINVAL;
    qeq_plan* pl = plan;
    int rc = QEQ_EINVAL;
    if (pos && sigma && J && chi && q) {
        pl->tape_valid = false;   // the adjoint and the virial follow periodic solves only
        pl->np_valid = false;
        pl->ew_active = false;
        pl->pw_active = false;
        pl->geom_valid = false;
        pl->spc_active = false;
        rc = np_setup(pl, n, pos, sigma, J, chi, q_tot);
        if (rc == QEQ_OK) {
            pl->direct = true;
            pl->fdst = pl->forces_s;
            bool conv = false;
            rc = cg_run(pl, q0, q, energies, forces, &conv);
            if (rc == QEQ_OK) rc = cg_status(pl, conv, stats);
            pl->np_valid = rc >= 0;
        }
    }
    if (rc < 0 && stats) {
        memset(stats, 0, sizeof(*stats));
        stats->status = rc;
    }
    return rc;
}

int qeq_element_potentials(qeq_plan* plan, const int32_t* species, int32_t n_elem, double* gamma) {
    if (!plan) return QEQ_EINVAL;
    return element_potentials_impl(plan, species, n_elem, gamma);
}

int qeq_matvec(qeq_plan* plan, int32_t n, const double* pos, const double* cell, const double* sigma,
               const double* v, double* y, int32_t parts) {
    if (!plan || !pos || !sigma || !v || !y) return QEQ_EINVAL;
    if (parts < 0 || parts > 15) return QEQ_EINVAL;
    qeq_plan* pl = plan;
    pl->tape_valid = false;
    pl->direct = false;
    pl->ew_active = false;
    pl->pw_active = false;
    pl->geom_valid = false;   // the operator parts below differ from a solve's
    QEQ_TRY(prepare(pl, n, cell, 0.0));
    QEQ_TRY(setup_geometry(pl, pos, sigma, nullptr, nullptr));
    pl->kp.parts = parts;
    QEQ_TRY(launch_matvec_io(pl, v, nullptr, 0));
    // the CG product's mesh path (fused interpolation where it applies)
    bool partials = false;
    if (parts & QEQ_PART_RECIP) QEQ_TRY(launch_mesh_cg(pl, pl->pvec, nullptr, &partials));
    QEQ_TRY(launch_interp(pl, pl->pvec, pl->y, QEQ_MODE_MATVEC, 0, partials ? pl->mpart : nullptr));
    QEQ_TRY(launch_matvec_io(pl, nullptr, y, 1));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    pl->kp.parts = 15;
    return QEQ_OK;
}

int qeq_use_graphs(qeq_plan* plan, int32_t enable) {
    if (plan && plan->stream) (void)hipStreamSynchronize(plan->stream);
    if (!plan) return QEQ_EINVAL;
    plan->use_graphs = enable != 0;
    if (!plan->use_graphs) drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_spectral_preconditioner(qeq_plan* plan, double k_cut) {
    if (!plan || !(k_cut == k_cut)) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->spc_kc = k_cut > 0.0 ? k_cut : 0.0;
    plan->spc_active = false;
    plan->tape_valid = false;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_ewald(qeq_plan* plan, int32_t enable) {
    if (!plan) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->ewald = enable != 0;
    if (plan->ewald) plan->planewave = false;
    plan->tape_valid = false;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_sqnm(qeq_plan* plan, int32_t enable, int32_t history) {
    if (!plan) return QEQ_EINVAL;
    if (history == 0) history = 10;
    if (enable && (history < 1 || history > 16)) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->sqnm = enable != 0;
    if (plan->sqnm && history != plan->sq_m) {
        sqnm_free(plan);
        plan->sq_m = history;
    }
    return QEQ_OK;
}

int qeq_use_planewave(qeq_plan* plan, int32_t enable, double support) {
    if (!plan) return QEQ_EINVAL;
    if (support == 0.0) support = 6.0;
    if (enable && !(support >= 3.0 && support <= 12.0)) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->planewave = enable != 0;
    if (plan->planewave) {
        plan->ewald = false;
        plan->pw_support = support;
    }
    plan->tape_valid = false;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_fused_inverse(qeq_plan* plan, int32_t enable) {
    if (!plan) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->fused_inverse = enable != 0;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_fused_forward(qeq_plan* plan, int32_t enable) {
    if (!plan) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->fused_forward = enable != 0;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_set_tiles(qeq_plan* plan, int32_t spread_rows, int32_t tile_rows, int32_t fft_rows) {
    if (!plan) return QEQ_EINVAL;
    const int v[3] = {spread_rows, tile_rows, fft_rows};
    for (int a = 0; a < 3; ++a) {
        const int t = v[a];
        const bool pow2 = t > 0 && (t & (t - 1)) == 0;
        // spread tiles may also be 12 or 24 rows (compiled widths only; the
        // launch refuses others with QEQ_EPLAN)
        const bool even_spread = a == 0 && (t == 12 || t == 24);
        if (t != 0 && !((pow2 || even_spread) && t >= (a == 2 ? 1 : 4) && t <= 32)) return QEQ_EINVAL;
    }
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    for (int a = 0; a < 3; ++a) plan->tile_set[a] = v[a];
    plan->geom_valid = false;
    plan->tape_valid = false;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_use_fused_interp(qeq_plan* plan, int32_t enable) {
    if (!plan) return QEQ_EINVAL;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    plan->fused_interp = enable != 0;
    drop_graph(plan);
    return QEQ_OK;
}

int qeq_time_kernel(qeq_plan* plan, int32_t kind, int32_t reps, double* avg_us) {
    if (!plan || !avg_us || reps < 1) return QEQ_EINVAL;
    const bool direct = kind == PK_COUNT;   // the isolated solve's pair-sum product
    if (direct ? !(plan->direct && plan->np_valid)
               : (!plan->tape_valid || (kind != PK_SPREAD_R2C && kind != PK_C2R)))
        return QEQ_EINVAL;
    qeq_plan* pl = plan;
    auto stage = [&]() {
        return direct ? launch_np_matvec(pl, pl->q, pl->y, QEQ_MODE_MATVEC) : launch_mesh_stage(pl, kind, pl->q);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QEQ_HIP(hipEventCreate(&e0));
    int rc = qeq_check(hipEventCreate(&e1));
    const unsigned mask = pl->prof_mask;
    pl->prof_mask = 0;
    if (rc == QEQ_OK) rc = stage();   // warm caches and code
    if (rc == QEQ_OK) rc = qeq_check(hipEventRecord(e0, pl->stream));
    for (int r = 0; r < reps && rc == QEQ_OK; ++r) rc = stage();
    if (rc == QEQ_OK) rc = qeq_check(hipEventRecord(e1, pl->stream));
    if (rc == QEQ_OK) rc = qeq_check(hipEventSynchronize(e1));
    float ms = 0.f;
    if (rc == QEQ_OK) rc = qeq_check(hipEventElapsedTime(&ms, e0, e1));
    pl->prof_mask = mask;
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == QEQ_OK) *avg_us = 1e3 * (double)ms / reps;
    return rc;
}

int qeq_profile(qeq_plan* plan, uint32_t kind_mask) {
    if (!plan) return QEQ_EINVAL;
    plan->prof_mask = kind_mask & ((1u << PK_COUNT) - 1u);
    return QEQ_OK;
}

int qeq_profile_read(qeq_plan* plan, double* total_ms, int64_t* launches, int32_t n_kinds,
                     int32_t reset) {
    if (!plan || n_kinds < 0) return QEQ_EINVAL;
    if (plan->stream) QEQ_HIP(hipStreamSynchronize(plan->stream));
    prof_flush(plan, 1 << 30);
    for (int k = 0; k < n_kinds && k < PK_COUNT; ++k) {
        if (total_ms) total_ms[k] = plan->prof_ms[k];
        if (launches) launches[k] = plan->prof_n[k];
    }
    if (reset) {
        for (int k = 0; k < PK_COUNT; ++k) {
            plan->prof_ms[k] = 0.0;
            plan->prof_n[k] = 0;
        }
    }
    return PK_COUNT;
}

int qeq_descriptors(qeq_plan* plan, int32_t n, const double* pos, const double* cell, const double* sigma,
                    const double* weights, int32_t n_feat, const double* centers, double width, double r_cut,
                    float* G) {
    if (!plan || !centers || !G) return QEQ_EINVAL;
    qeq_plan* pl = plan;
    if (pos) {
        if (!sigma) return QEQ_EINVAL;
        pl->tape_valid = false;   // the geometry set-up below replaces the solve's tape
        pl->geom_valid = false;
        pl->ew_active = false;
        pl->pw_active = false;
        QEQ_TRY(prepare(pl, n, cell, 0.0));
        QEQ_TRY(setup_geometry(pl, pos, sigma, nullptr, nullptr));
        pl->geom_valid = true;
    } else if (!pl->geom_valid || n != pl->kp.n) {
        return QEQ_EINVAL;   // no geometry of this size to reuse
    }
    QEQ_TRY(launch_descriptors(pl, weights, n_feat, centers, width, r_cut, G));
    QEQ_HIP(hipStreamSynchronize(pl->stream));
    return QEQ_OK;
}

int qeq_backward(qeq_plan* plan, const double* dL_dq, double dL_dEelec, double dL_dEqeq,
                 double* dL_dchi, double* dL_dJ, double* dL_dpos, qeq_stats* stats) {
    if (!plan) return QEQ_EINVAL;
    int rc = backward_impl(plan, dL_dq, dL_dEelec, dL_dEqeq, dL_dchi, dL_dJ, dL_dpos, stats);
    if (rc < 0 && stats) {
        memset(stats, 0, sizeof(*stats));
        stats->status = rc;
    }
    return rc;
}

int qeq_virial(qeq_plan* plan, double* virial) {
    if (!plan) return QEQ_EINVAL;
    return virial_impl(plan, virial);
}

const char* qeq_strerror(int code) {
    switch (code) {
        case QEQ_OK: return "success";
        case QEQ_NOT_CONVERGED: return "CG reached max_iter before the residual tolerance";
        case QEQ_EINVAL: return "invalid argument (n, J <= 0, sigma <= 0, non-finite input or singular cell)";
        case QEQ_ECELL: return "cell too skewed for the real-space cell list";
        case QEQ_ENOMEM: return "device allocation failed";
        case QEQ_EHIP: return "HIP runtime error";
        case QEQ_EPLAN: return "unsupported grid or spline order, or n larger than the plan";
        default: return "unknown status code";
    }
}

}  // extern "C"
