// Per-geometry setup: input staging and validation, spatial sort of atoms by
// grid column, B-spline weights, the real-space cell list and pair list, and
// the per-atom mesh self-interaction correction.
#include <math.h>

#include "internal.h"

namespace {

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

__device__ __forceinline__ void frac_coords(const KParams& k, const double* x, double* s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = x[0] * k.Hinv[0 * 3 + a] + x[1] * k.Hinv[1 * 3 + a] + x[2] * k.Hinv[2 * 3 + a];
        v -= floor(v);
        if (!(v >= 0.0 && v < 1.0)) v = 0.0;   // v == 1 after rounding, or non-finite input
        s[a] = v;
    }
}

__device__ __forceinline__ int grid_home(double s, int K) {
    int h = (int)floor(s * (double)K);
    return h < 0 ? 0 : (h >= K ? K - 1 : h);
}

// ---------------------------------------------------------------------------
// Stage (original order): validate, fractional coordinates, grid-column key.
// ---------------------------------------------------------------------------
__global__ void k_stage(KParams k, const double* __restrict__ pos, const double* __restrict__ sigma,
                        const double* __restrict__ J, const double* __restrict__ chi,
                        int* __restrict__ key, int* __restrict__ bin_count, CgScalars* sc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k.n) return;
    double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double jj = J ? J[i] : 1.0, ch = chi ? chi[i] : 0.0;
    bool ok = finite_d(x[0]) && finite_d(x[1]) && finite_d(x[2]) && finite_d(ch) &&
              sigma[i] > 0.0 && jj > 0.0 && finite_d(sigma[i]) && finite_d(jj);
    if (!ok) atomicOr(&sc->err, QEQ_ERRBIT_INPUT);
    double s[3];
    frac_coords(k, x, s);
    int h1 = grid_home(s[0], k.K1), h2 = grid_home(s[1], k.K2);
    int kk = h1 * k.K2 + h2;
    key[i] = kk;
    atomicAdd(&bin_count[kk], 1);
}

__global__ void k_scatter(int n, const int* __restrict__ key, const int* __restrict__ start,
                          int* __restrict__ fill, int* __restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int kk = key[i];
    int slot = start[kk] + atomicAdd(&fill[kk], 1);
    perm[slot] = i;
}

// Deterministic order inside each bucket: ascending index.
__global__ void k_bucket_sort(int nb, const int* __restrict__ start, int* __restrict__ v) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int lo = start[b], hi = start[b + 1];
    for (int a = lo + 1; a < hi; ++a) {
        int x = v[a];
        int c = a - 1;
        while (c >= lo && v[c] > x) {
            v[c + 1] = v[c];
            --c;
        }
        v[c + 1] = x;
    }
}

// Exclusive scan of m ints in three launches: per-block totals of 1024-element
// chunks, a one-block scan of those totals, then each chunk scanned with its
// offset.  out[m] = total.
constexpr int SCAN_CHUNK = 1024;

__global__ __launch_bounds__(256) void k_scan_totals(const int* __restrict__ in, int m, int* __restrict__ tot) {
    const int base = blockIdx.x * SCAN_CHUNK;
    int v = 0;
    for (int t = threadIdx.x; t < SCAN_CHUNK; t += 256) v += base + t < m ? in[base + t] : 0;
    double d[1] = {(double)v};
    block_sum<1>(d);
    if (threadIdx.x == 0) tot[blockIdx.x] = (int)d[0];
}

__global__ __launch_bounds__(256) void k_scan_chunks(const int* __restrict__ in, int m, const int* __restrict__ tot,
                                                    int nchunk, int* __restrict__ out) {
    __shared__ int part[256];
    __shared__ int offset;
    const int t = threadIdx.x;
    {
        double o[1] = {0.0};
        for (int b = t; b < (int)blockIdx.x; b += 256) o[0] += (double)tot[b];
        block_sum<1>(o);
        if (t == 0) offset = (int)o[0];
    }
    // 4 consecutive elements per thread
    const int base = blockIdx.x * SCAN_CHUNK + 4 * t;
    int v[4], s = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        v[u] = base + u < m ? in[base + u] : 0;
        s += v[u];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int run = offset + part[t] - s;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (base + u < m) out[base + u] = run;
        run += v[u];
    }
    if (blockIdx.x == nchunk - 1 && t == 255) out[m] = offset + part[255];
}

// Exclusive scan of m ints into out[0..m], out[m] = total; one block.
__global__ void k_scan(const int* __restrict__ in, int* __restrict__ out, int m) {
    __shared__ int part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    int chunk = (m + nt - 1) / nt;
    int lo = t * chunk, hi = min(m, lo + chunk);
    int s = 0;
    for (int a = lo; a < hi; ++a) s += in[a];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int a = lo; a < hi; ++a) {
        out[a] = run;
        run += in[a];
    }
    if (t == nt - 1) out[m] = part[t];
}

// ---------------------------------------------------------------------------
// Gather (sorted order): copy per-atom data, B-spline weights, cell key.
// ---------------------------------------------------------------------------
__global__ void k_gather(KParams k, const double* __restrict__ pos, const double* __restrict__ sigma,
                         const double* __restrict__ J, const double* __restrict__ chi,
                         const int* __restrict__ perm, double* __restrict__ frac, int* __restrict__ home,
                         float* __restrict__ wts, float* __restrict__ dwts, double* __restrict__ sig_s,
                         double* __restrict__ J_s, double* __restrict__ chi_s,
                         double* __restrict__ chi_raw_s, double* __restrict__ dself,
                         double* __restrict__ dinv, int* __restrict__ cell_count,
                         double* __restrict__ part) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (s < k.n) {
        int i = perm[s];
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double f[3];
        frac_coords(k, x, f);
        int Kd[3] = {k.K1, k.K2, k.K3};
        int h[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            frac[3 * s + a] = f[a];
            double u = f[a] * (double)Kd[a];
            h[a] = grid_home(f[a], Kd[a]);
            double w = u - (double)h[a];
            double c[QEQ_MAXP], dc[QEQ_MAXP];
            bspline_weights<double>(w, k.p, c, dc);
            for (int kk = 0; kk < QEQ_MAXP; ++kk) {
                wts[(s * 3 + a) * QEQ_MAXP + kk] = kk < k.p ? (float)c[kk] : 0.f;
                dwts[(s * 3 + a) * QEQ_MAXP + kk] = kk < k.p ? (float)dc[kk] : 0.f;
            }
        }
        int c[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = (int)(f[a] * (double)k.nc[a]);
            if (c[a] >= k.nc[a]) c[a] = k.nc[a] - 1;
        }
        int ck = (c[0] * k.nc[1] + c[1]) * k.nc[2] + c[2];
        home[4 * s + 0] = h[0];
        home[4 * s + 1] = h[1];
        home[4 * s + 2] = h[2];
        home[4 * s + 3] = ck;
        atomicAdd(&cell_count[ck], 1);
        double sg = sigma[i], jj = J ? J[i] : 1.0, c0 = chi ? chi[i] : 0.0;
        double ce = c0 + k.bg_pref * k.q_tot * sg * sg;
        sig_s[s] = sg;
        J_s[s] = jj;
        chi_s[s] = ce;
        chi_raw_s[s] = c0;
        const double rsqpi = 0.56418958354775628695;   // 1/sqrt(pi)
        dself[s] = rsqpi / sg - 0.79788456080286535588 / k.eta;   // - sqrt(2/pi)/eta
        dinv[s] = 1.0 / (jj + rsqpi / sg);
        acc[0] = ce;
        acc[1] = dinv[s];
    }
    block_sum<3>(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x * QEQ_NPART + 0] = acc[0];
        part[blockIdx.x * QEQ_NPART + 1] = acc[1];
    }
}

// ||P chi_eff|| needs the mean first: two passes over chi_eff.
__global__ void k_chi_norm(int n, const double* __restrict__ chi_s, double* __restrict__ part,
                           int nparts, double* __restrict__ part_out) {
    double tot[2];
    // reduce first-pass partials (layout stride QEQ_NPART)
    __shared__ double sh_mean;
    {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nparts; b += blockDim.x) v[0] += part[b * QEQ_NPART];
        block_sum<1>(v);
        if (threadIdx.x == 0) sh_mean = v[0] / (double)n;
        __syncthreads();
    }
    double mean = sh_mean;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    tot[0] = 0.0;
    tot[1] = 0.0;
    if (s < n) {
        double d = chi_s[s] - mean;
        tot[0] = d * d;
    }
    block_sum<2>(tot);
    if (threadIdx.x == 0) {
        part_out[blockIdx.x * QEQ_NPART + 0] = tot[0];
        part_out[blockIdx.x * QEQ_NPART + 1] = mean;
    }
}

__global__ void k_chi_finish(int n, const double* __restrict__ part1, const double* __restrict__ part2,
                             int nparts, CgScalars* sc) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        v[0] += part1[b * QEQ_NPART];
        v[1] += part2[b * QEQ_NPART];
        v[2] += part1[b * QEQ_NPART + 1];
    }
    block_sum<3>(v);
    if (threadIdx.x == 0) {
        sc->chi_sum = v[0];
        sc->chi_norm = sqrt(v[1]);
        sc->dinv_sum = v[2];
    }
}

__global__ void k_cell_scatter(int n, const int* __restrict__ home, const int* __restrict__ start,
                               int* __restrict__ fill, int* __restrict__ atoms) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int ck = home[4 * s + 3];
    atoms[start[ck] + atomicAdd(&fill[ck], 1)] = s;
}

// One wave per atom i: the lanes share the cells of the stencil around i's
// cell (lane l takes stencil cells l, l + 64, ...), count or write the pairs
// found there; a wave prefix sum gives each lane its slice of row i, so the
// row order is fixed (lane-major, cells in stencil order, atoms in cell order).
template <bool FILL>
__global__ __launch_bounds__(QEQ_BLOCK) void k_pairs(KParams k, const double* __restrict__ frac,
                                                    const int* __restrict__ home, const double* __restrict__ sig,
                                                    const int* __restrict__ cell_start,
                                                    const int* __restrict__ cell_atoms, int* __restrict__ rowcnt,
                                                    const int* __restrict__ rowptr, int* __restrict__ col,
                                                    float* __restrict__ kval, float4* __restrict__ pdr,
                                                    long long cap, int* __restrict__ lanecnt) {
    // FILL stages a row of up to PBUF pairs in this wave's LDS slice and
    // evaluates the FP64 kernel values afterwards with one pair per lane
    // (inside the stencil loop the divergent lanes would run the erf pair
    // once per step); longer rows evaluate them in place.  The staged
    // distance is kept in FP64, so staged and in-place rows evaluate the
    // kernel at the same argument.
    constexpr int PBUF = 128;
    __shared__ float4 st_d[FILL ? (QEQ_BLOCK / 64) * PBUF : 1];
    __shared__ double st_r[FILL ? (QEQ_BLOCK / 64) * PBUF : 1];
    __shared__ int st_j[FILL ? (QEQ_BLOCK / 64) * PBUF : 1];
    const int lane = threadIdx.x & 63;
    const int i = (xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
    if (i >= k.n) return;   // uniform across the wave
    // the host sized the pair arrays before the count was known: a row that
    // would run past the capacity is left out (the host reads the count,
    // grows the arrays and fills again)
    if (FILL && rowptr[i + 1] > cap) return;
    const int sbase = (threadIdx.x >> 6) * PBUF;
    const bool staged = FILL && rowptr[i + 1] - rowptr[i] <= PBUF;
    int loff = 0;
    const double si[3] = {frac[3 * i], frac[3 * i + 1], frac[3 * i + 2]};
    const int ck = home[4 * i + 3];
    const int c3 = ck % k.nc[2];
    const int c2 = (ck / k.nc[2]) % k.nc[1];
    const int c1 = ck / (k.nc[2] * k.nc[1]);
    const double sgi = sig[i];
    const int w2 = 2 * k.ns[1] + 1, w3 = 2 * k.ns[2] + 1;
    const int nst = (2 * k.ns[0] + 1) * w2 * w3;
    int off = 0;
    if (FILL) {
        // this lane's slice of the row, from the counts that the count pass
        // took over the same stencil walk
        const int c = lanecnt[(size_t)i * 64 + lane];
        int incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        off = rowptr[i] + incl - c;
        loff = incl - c;
    }
    {
        // count (with the lane's count kept for the fill) or write
        int cnt = 0;
        for (int t = lane; t < nst; t += 64) {
            const int d3 = t % w3 - k.ns[2], d2 = (t / w3) % w2 - k.ns[1], d1 = t / (w3 * w2) - k.ns[0];
            const int r1 = c1 + d1, r2 = c2 + d2, r3 = c3 + d3;
            const int x1 = wrap_idx(r1, k.nc[0]), x2 = wrap_idx(r2, k.nc[1]), x3 = wrap_idx(r3, k.nc[2]);
            const int sh1 = (r1 - x1) / k.nc[0], sh2 = (r2 - x2) / k.nc[1], sh3 = (r3 - x3) / k.nc[2];
            const int cell = (x1 * k.nc[1] + x2) * k.nc[2] + x3;
            const bool home_img = (sh1 == 0 && sh2 == 0 && sh3 == 0);
            for (int u = cell_start[cell]; u < cell_start[cell + 1]; ++u) {
                const int j = cell_atoms[u];
                if (home_img && j == i) continue;
                const double ds0 = frac[3 * j] + sh1 - si[0];
                const double ds1 = frac[3 * j + 1] + sh2 - si[1];
                const double ds2 = frac[3 * j + 2] + sh3 - si[2];
                // d = r_j(image) - r_i, Cartesian (row vector ds times H)
                const double dx = ds0 * k.H[0] + ds1 * k.H[3] + ds2 * k.H[6];
                const double dy = ds0 * k.H[1] + ds1 * k.H[4] + ds2 * k.H[7];
                const double dz = ds0 * k.H[2] + ds1 * k.H[5] + ds2 * k.H[8];
                const double r2v = dx * dx + dy * dy + dz * dz;
                if (r2v >= k.rc2) continue;
                if (FILL) {
                    if (staged) {
                        // r_i - r_j(image) for the force, the FP64 distance beside it
                        st_j[sbase + loff] = j;
                        st_d[sbase + loff] = make_float4((float)(-dx), (float)(-dy), (float)(-dz), 0.f);
                        st_r[sbase + loff] = sqrt(r2v);
                        ++loff;
                    } else {
                        const double sj = sig[j];
                        double K, dKr;
                        pair_kernel(sqrt(r2v), sqrt(sgi * sgi + sj * sj), k.eta, &K, &dKr);
                        col[off] = j;
                        kval[off] = (float)K;
                        pdr[off] = make_float4((float)(-dx), (float)(-dy), (float)(-dz), (float)dKr);
                        ++off;
                    }
                }
                ++cnt;
            }
        }
        if (!FILL) {
            lanecnt[(size_t)i * 64 + lane] = cnt;
            int incl = cnt;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane == 63) rowcnt[i] = incl;
        }
    }
    if (staged) {
        // the other lanes' LDS writes before the reads below (one wave)
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        const int e0 = rowptr[i], rl = rowptr[i + 1] - e0;
        for (int e = lane; e < rl; e += 64) {
            const int j = st_j[sbase + e];
            const float4 d = st_d[sbase + e];
            const double sj = sig[j];
            double K, dKr;
            pair_kernel(st_r[sbase + e], sqrt(sgi * sgi + sj * sj), k.eta, &K, &dKr);
            col[e0 + e] = j;
            kval[e0 + e] = (float)K;
            pdr[e0 + e] = make_float4(d.x, d.y, d.z, (float)dKr);
        }
    }
}

// ---------------------------------------------------------------------------
// Mesh self-interaction correction.  The mesh reproduces the reciprocal self
// term C_eta of atom i as theta_i^T Theta theta_i, which depends on where the
// atom sits inside its grid cell; c_i = C_eta - theta_i^T Theta theta_i is
// added to the diagonal (and its position derivative to the force), so the
// self term becomes exact.  With separable spline weights W_a,
//   theta_i^T Theta theta_i = sum_d Theta(d) R_1(d_1) R_2(d_2) R_3(d_3),
//   R_a(d) = sum_{k' - k = d} W_a[k] W_a[k'],  |d_a| <= p - 1.
// ---------------------------------------------------------------------------
__global__ void k_theta_extract(KParams k, const float* __restrict__ grid, double* __restrict__ tab) {
    int np = 2 * k.p - 1;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * np * np) return;
    int d3 = t % np - (k.p - 1);
    int d2 = (t / np) % np - (k.p - 1);
    int d1 = t / (np * np) - (k.p - 1);
    int g1 = wrap_idx(d1, k.K1), g2 = wrap_idx(d2, k.K2), g3 = wrap_idx(d3, k.K3);
    tab[t] = (double)grid[((size_t)g1 * k.K2 + g2) * k.K3 + g3];
}

template <int PC>
__global__ void k_selfcorr(KParams k, const double* __restrict__ frac, const double* __restrict__ tab_g,
                           double* __restrict__ dself, double* __restrict__ selfgrad) {
    // the table is read by every atom: stage it in LDS
    __shared__ double tab[(2 * QEQ_MAXP - 1) * (2 * QEQ_MAXP - 1) * (2 * QEQ_MAXP - 1)];
    const int np = 2 * k.p - 1;
    for (int t = threadIdx.x; t < np * np * np; t += blockDim.x) tab[t] = tab_g[t];
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k.n) return;
    const double u[3] = {frac[3 * i] * (double)k.K1, frac[3 * i + 1] * (double)k.K2,
                         frac[3 * i + 2] * (double)k.K3};
    double s, g[3];
    mesh_self_term<PC>(u, k.p, tab, &s, g);
    dself[i] += k.c_eta - s;
    selfgrad[3 * i + 0] = g[0];
    selfgrad[3 * i + 1] = g[1];
    selfgrad[3 * i + 2] = g[2];
}

// Virial of the self-correction: per atom theta_i^T dTheta_ab theta_i for the
// six strain components (one table staged in LDS at a time), weighted by q^2;
// also sum q^2 and sum q sigma^2 for the C_eta and background terms.
template <int PC>
__global__ __launch_bounds__(QEQ_BLOCK) void k_self_strain(KParams k, const double* __restrict__ frac,
                                                          const double* __restrict__ tabs,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ sig,
                                                          double* __restrict__ part) {
    __shared__ double tab[(2 * QEQ_MAXP - 1) * (2 * QEQ_MAXP - 1) * (2 * QEQ_MAXP - 1)];
    const int np = 2 * k.p - 1;
    const int np3 = np * np * np;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < k.n;
    double acc[QEQ_NPART];
#pragma unroll
    for (int t = 0; t < QEQ_NPART; ++t) acc[t] = 0.0;
    const double qi = act ? q[i] : 0.0;
    if (tabs) {
        double u[3] = {0.0, 0.0, 0.0};
        if (act) {
            u[0] = frac[3 * i] * (double)k.K1;
            u[1] = frac[3 * i + 1] * (double)k.K2;
            u[2] = frac[3 * i + 2] * (double)k.K3;
        }
        for (int comp = 0; comp < 6; ++comp) {
            __syncthreads();
            for (int t = threadIdx.x; t < np3; t += blockDim.x) tab[t] = tabs[(size_t)comp * np3 + t];
            __syncthreads();
            if (act) {
                double s, g[3];
                mesh_self_term<PC>(u, k.p, tab, &s, g);
                acc[comp] = qi * qi * s;
            }
        }
    }
    if (act) {
        acc[6] = qi * qi;
        acc[7] = qi * sig[i] * sig[i];
    }
    block_sum<QEQ_NPART>(acc);
    if (threadIdx.x == 0)
        for (int t = 0; t < QEQ_NPART; ++t) part[(size_t)blockIdx.x * QEQ_NPART + t] = acc[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_scan(qeq_plan* pl, const int* in, int* out, int m) {
    const int nchunk = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nchunk <= 4) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, pl->stream, in, out, m);
        return qeq_check(hipGetLastError());
    }
    if ((size_t)nchunk > pl->scan_cap) {
        if (pl->scan_tmp) (void)hipFree(pl->scan_tmp);
        pl->scan_tmp = nullptr;
        pl->scan_cap = 0;
        if (hipMalloc((void**)&pl->scan_tmp, sizeof(int) * (size_t)nchunk) != hipSuccess) return QEQ_ENOMEM;
        pl->scan_cap = (size_t)nchunk;
    }
    hipLaunchKernelGGL(k_scan_totals, dim3(nchunk), dim3(256), 0, pl->stream, in, m, pl->scan_tmp);
    hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(256), 0, pl->stream, in, m, pl->scan_tmp, nchunk, out);
    return qeq_check(hipGetLastError());
}

// The set-up's bin and cell counters and the CG scalars, zeroed in one launch
// (separate memsets would each cost the host a call while the GPU waits).
__global__ void k_setup_clear(int* __restrict__ sc_words, int nsc, int* __restrict__ bc, int* __restrict__ bf,
                              int nbins, int* __restrict__ cc, int* __restrict__ cf, int ncells) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nsc) sc_words[t] = 0;
    if (t < nbins) {
        bc[t] = 0;
        bf[t] = 0;
    }
    if (t < ncells) {
        cc[t] = 0;
        cf[t] = 0;
    }
}

int launch_setup_clear(qeq_plan* pl) {
    const KParams& k = pl->kp;
    static_assert(sizeof(CgScalars) % sizeof(int) == 0, "CgScalars clears as ints");
    const int nsc = (int)(sizeof(CgScalars) / sizeof(int));
    const int nbins = k.K1 * k.K2 + 1, ncells = k.nc[0] * k.nc[1] * k.nc[2] + 1;
    const int m = std::max(nsc, std::max(nbins, ncells));
    hipLaunchKernelGGL(k_setup_clear, dim3((m + QEQ_BLOCK - 1) / QEQ_BLOCK), dim3(QEQ_BLOCK), 0, pl->stream,
                       reinterpret_cast<int*>(pl->sc), nsc, pl->bin_count, pl->bin_fill, nbins, pl->cell_count,
                       pl->cell_fill, ncells);
    return qeq_check(hipGetLastError());
}

int launch_stage(qeq_plan* pl, const double* pos, const double* sigma, const double* J,
                 const double* chi) {
    const KParams& k = pl->kp;
    hipLaunchKernelGGL(k_stage, dim3(nblocks(k.n)), dim3(QEQ_BLOCK), 0, pl->stream, k, pos, sigma,
                       J, chi, pl->key, pl->bin_count, pl->sc);
    return qeq_check(hipGetLastError());
}

int launch_sort_bins(qeq_plan* pl) {
    const KParams& k = pl->kp;
    int nb = k.K1 * k.K2;
    QEQ_TRY(launch_scan(pl, pl->bin_count, pl->bin_start, nb));
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(k.n)), dim3(QEQ_BLOCK), 0, pl->stream, k.n, pl->key,
                       pl->bin_start, pl->bin_fill, pl->perm);
    hipLaunchKernelGGL(k_bucket_sort, dim3(nblocks(nb)), dim3(QEQ_BLOCK), 0, pl->stream, nb,
                       pl->bin_start, pl->perm);
    return qeq_check(hipGetLastError());
}

int launch_gather(qeq_plan* pl, const double* pos, const double* sigma, const double* J,
                  const double* chi) {
    const KParams& k = pl->kp;
    int nb = nblocks(k.n);
    double* part1 = pl->part;
    double* part2 = pl->part + (size_t)pl->nblk_max * QEQ_NPART;
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, k, pos, sigma, J, chi,
                       pl->perm, pl->frac, pl->home, pl->wts, pl->dwts, pl->sig, pl->Jv, pl->chi,
                       pl->chi_raw, pl->dself, pl->dinv, pl->cell_count, part1);
    hipLaunchKernelGGL(k_chi_norm, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, k.n, pl->chi, part1, nb,
                       part2);
    hipLaunchKernelGGL(k_chi_finish, dim3(1), dim3(QEQ_BLOCK), 0, pl->stream, k.n, part1, part2, nb,
                       pl->sc);
    return qeq_check(hipGetLastError());
}

// ||P b|| and sum b of a right-hand side whose partial sums (slot 0: sum b,
// slot 1: sum 1/D) are already in the first partial buffer.
int launch_rhs_norm(qeq_plan* pl, const double* b) {
    const int nb = nblocks(pl->kp.n);
    double* part1 = pl->part;
    double* part2 = pl->part + (size_t)pl->nblk_max * QEQ_NPART;
    hipLaunchKernelGGL(k_chi_norm, dim3(nb), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp.n, b, part1, nb, part2);
    hipLaunchKernelGGL(k_chi_finish, dim3(1), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp.n, part1, part2, nb,
                       pl->sc);
    return qeq_check(hipGetLastError());
}

int launch_cells_and_pairs(qeq_plan* pl) {
    const KParams& k = pl->kp;
    int ncell = k.nc[0] * k.nc[1] * k.nc[2];
    QEQ_TRY(launch_scan(pl, pl->cell_count, pl->cell_start, ncell));
    hipLaunchKernelGGL(k_cell_scatter, dim3(nblocks(k.n)), dim3(QEQ_BLOCK), 0, pl->stream, k.n,
                       pl->home, pl->cell_start, pl->cell_fill, pl->cell_atoms);
    hipLaunchKernelGGL(k_bucket_sort, dim3(nblocks(ncell)), dim3(QEQ_BLOCK), 0, pl->stream, ncell,
                       pl->cell_start, pl->cell_atoms);
    const int pair_blocks = nblocks(k.n * 64);   // one wave per atom
    hipLaunchKernelGGL(k_pairs<false>, dim3(pair_blocks), dim3(QEQ_BLOCK), 0, pl->stream, k,
                       pl->frac, pl->home, pl->sig, pl->cell_start, pl->cell_atoms, pl->rowcnt,
                       pl->rowptr, pl->col, pl->kval, pl->pdr, (long long)0, pl->lanecnt);
    QEQ_TRY(launch_scan(pl, pl->rowcnt, pl->rowptr, k.n));
    // the total goes to the host with the set-up's error flag (one read-back
    // for both, in setup_geometry); until then the arrays keep their size, or
    // on a plan's first set-up the size a uniform density predicts
    if (pl->nnz_cap == 0) {
        const double vol = fabs(k.vol);
        const double mean = (double)k.n / vol * 4.0 / 3.0 * 3.14159265358979 * k.rc * k.rc * k.rc;
        QEQ_TRY(grow_pairs(pl, (size_t)((double)k.n * (mean * 1.15 + 8.0)) + 1024));
    }
    QEQ_HIP(hipMemcpyAsync(pl->nnz_host, pl->rowptr + k.n, sizeof(int), hipMemcpyDeviceToHost, pl->stream));
    return launch_pair_fill(pl);
}

int launch_pair_fill(qeq_plan* pl) {
    const KParams& k = pl->kp;
    hipLaunchKernelGGL(k_pairs<true>, dim3(nblocks(k.n * 64)), dim3(QEQ_BLOCK), 0, pl->stream, k,
                       pl->frac, pl->home, pl->sig, pl->cell_start, pl->cell_atoms, pl->rowcnt,
                       pl->rowptr, pl->col, pl->kval, pl->pdr, (long long)pl->nnz_cap, pl->lanecnt);
    return qeq_check(hipGetLastError());
}

int grow_pairs(qeq_plan* pl, size_t cap) {
    if (cap <= pl->nnz_cap) return QEQ_OK;
    if (pl->col) (void)hipFree(pl->col);
    if (pl->kval) (void)hipFree(pl->kval);
    if (pl->pdr) (void)hipFree(pl->pdr);
    pl->col = nullptr;
    pl->kval = nullptr;
    pl->pdr = nullptr;
    pl->nnz_cap = 0;
    if (hipMalloc(&pl->col, cap * sizeof(int)) != hipSuccess || hipMalloc(&pl->kval, cap * sizeof(float)) != hipSuccess ||
        hipMalloc(&pl->pdr, cap * sizeof(float4)) != hipSuccess)
        return QEQ_ENOMEM;
    debug_poison(pl->kval, cap * sizeof(float));
    debug_poison(pl->pdr, cap * sizeof(float4));
    pl->nnz_cap = cap;
    return QEQ_OK;
}

int launch_theta(qeq_plan* pl) {
    QEQ_TRY(launch_write_green(pl));
    QEQ_TRY(launch_mesh_inverse(pl));
    int np = 2 * pl->kp.p - 1;
    hipLaunchKernelGGL(k_theta_extract, dim3(nblocks(np * np * np)), dim3(QEQ_BLOCK), 0, pl->stream,
                       pl->kp, pl->grid_r, pl->theta_tab);
    return qeq_check(hipGetLastError());
}

int launch_selfcorr(qeq_plan* pl) {
    if (pl->kp.p == 6)
        hipLaunchKernelGGL(k_selfcorr<6>, dim3(nblocks(pl->kp.n)), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp,
                           pl->frac, pl->theta_tab, pl->dself, pl->selfgrad);
    else
        hipLaunchKernelGGL(k_selfcorr<0>, dim3(nblocks(pl->kp.n)), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp,
                           pl->frac, pl->theta_tab, pl->dself, pl->selfgrad);
    return qeq_check(hipGetLastError());
}

int launch_theta_strain(qeq_plan* pl, double* tabs) {
    const int np = 2 * pl->kp.p - 1;
    const int np3 = np * np * np;
    for (int comp = 0; comp < 6; ++comp) {
        QEQ_TRY(launch_write_green_strain(pl, comp));
        QEQ_TRY(launch_mesh_inverse(pl));
        hipLaunchKernelGGL(k_theta_extract, dim3(nblocks(np3)), dim3(QEQ_BLOCK), 0, pl->stream, pl->kp,
                           pl->grid_r, tabs + (size_t)comp * np3);
        QEQ_TRY(qeq_check(hipGetLastError()));
    }
    return QEQ_OK;
}

int launch_self_strain(qeq_plan* pl, const double* tabs, double* part) {
    const KParams& k = pl->kp;
    if (k.p == 6)
        hipLaunchKernelGGL(k_self_strain<6>, dim3(nblocks(k.n)), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->frac, tabs,
                           pl->q, pl->sig, part);
    else
        hipLaunchKernelGGL(k_self_strain<0>, dim3(nblocks(k.n)), dim3(QEQ_BLOCK), 0, pl->stream, k, pl->frac, tabs,
                           pl->q, pl->sig, part);
    return qeq_check(hipGetLastError());
}
