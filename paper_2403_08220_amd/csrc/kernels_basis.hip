// KLE basis of the grid Matern prior (Sec. 4.2), Rao-Blackwellised posterior
// moments (the Gaussian lemma of Sec. 5.3) and the multichain ESS fraction (Sec. 6.2.2, eq. ess).
#include "dino_internal.hpp"

namespace dino {

// DCT-II mode k at node i of an n-point line: sqrt((2 - [k=0])/n) cos(pi k (i + 1/2)/n).
__device__ __forceinline__ double dct_q(int n, int k, int i) {
    const double scale = (k == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
    return scale * cos(M_PI * (double)k * ((double)i + 0.5) / (double)n);
}

// dec[p][j] = sqrt(lam_j) q_{k1_j}(i) q_{k2_j}(jy), p = jy*n + i.
__global__ void basis_dec_kernel(int n, int r, const int32_t* __restrict__ k1, const int32_t* __restrict__ k2,
                                 const double* __restrict__ lam, double* __restrict__ dec) {
    const long total = (long)n * n * r;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e % r);
        const long p = e / r;
        const int i = (int)(p % n), jy = (int)(p / n);
        dec[e] = sqrt(lam[j]) * dct_q(n, k1[j], i) * dct_q(n, k2[j], jy);
    }
}

// Q2[i][k] = q_k(i)^2.
__global__ void q2_kernel(int n, double* __restrict__ Q2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, k = e % n;
    const double q = dct_q(n, k, i);
    Q2[e] = q * q;
}

// T[i][k2] = sum_k1 Q2[i][k1] lamc[k1][k2]
__global__ void vp_stage1_kernel(int n, const double* __restrict__ Q2, const double* __restrict__ lamc,
                                 double* __restrict__ T) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, k2 = e % n;
    double acc = 0.0;
    for (int k1 = 0; k1 < n; ++k1) acc += Q2[i * n + k1] * lamc[k1 * n + k2];
    T[e] = acc;
}

// var_perp[jy*n + i] = sum_k2 T[i][k2] Q2[jy][k2]
__global__ void vp_stage2_kernel(int n, const double* __restrict__ Q2, const double* __restrict__ T,
                                 double* __restrict__ vp) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int jy = e / n, i = e % n;
    double acc = 0.0;
    for (int k2 = 0; k2 < n; ++k2) acc += T[i * n + k2] * Q2[jy * n + k2];
    vp[e] = acc;
}

// Q[i][k] = q_k(i).
__global__ void q_kernel(int n, double* __restrict__ Q) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    Q[e] = dct_q(n, e % n, e / n);
}

// One axis of the separable transform for nf fields of n x n values:
//     out[f][b][a] = sum_c in[f][a][c] Q[c][b]   (trans = 0)
//     out[f][b][a] = sum_c in[f][a][c] Q[b][c]   (trans = 1),
// i.e. the last axis is contracted with Q (or Q^T) and the two axes swap.
__global__ void sep_axis_kernel(int nf, int n, const double* __restrict__ in, const double* __restrict__ Q,
                                int trans, double* __restrict__ out) {
    const long nn = (long)n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const int b = e / n, a = e % n;
    for (int f = blockIdx.y; f < nf; f += gridDim.y) {  // the grid's y extent is capped at GRID_Y_MAX
        const double* row = in + f * nn + (long)a * n;
        double acc = 0.0;
        if (trans)
            for (int c = 0; c < n; ++c) acc += row[c] * Q[(long)b * n + c];
        else
            for (int c = 0; c < n; ++c) acc += row[c] * Q[(long)c * n + b];
        out[f * nn + e] = acc;
    }
}

// KLE position t holds mode perm[t] = k1 n + k2; the transformed grid is laid out
// [k2][k1]. Encode: z_t = G[k2][k1] / sqrt(lambda_t); decode scatters G = z sqrt(lambda).
__global__ void kle_gather_kernel(int nf, int n, int r, const double* __restrict__ G, const int32_t* __restrict__ perm,
                                  const double* __restrict__ sqlam, double* __restrict__ x,
                                  double* __restrict__ zp) {
    const long nn = (long)n * n;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn) return;
    const int e = perm[t], k1 = e / n, k2 = e % n;
    for (int f = blockIdx.y; f < nf; f += gridDim.y) {  // the grid's y extent is capped at GRID_Y_MAX
        const double z = G[f * nn + (long)k2 * n + k1] / sqlam[t];
        if (t < r) {
            if (x) x[(long)f * r + t] = z;
        } else if (zp) {
            zp[(long)f * (nn - r) + (t - r)] = z;
        }
    }
}

__global__ void kle_scatter_kernel(int nf, int n, int r, const double* __restrict__ x, const double* __restrict__ zp,
                                   const int32_t* __restrict__ perm, const double* __restrict__ sqlam,
                                   double* __restrict__ G) {
    const long nn = (long)n * n;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn) return;
    const int e = perm[t], k1 = e / n, k2 = e % n;
    for (int f = blockIdx.y; f < nf; f += gridDim.y) {  // the grid's y extent is capped at GRID_Y_MAX
        const double z = (t < r) ? x[(long)f * r + t] : (zp ? zp[(long)f * (nn - r) + (t - r)] : 0.0);
        G[f * nn + (long)k2 * n + k1] = z * sqlam[t];
    }
}

// Dense basis: out[f][p] = (w ? w[f][p] : 0) + sum_j (a[f][j] - (c ? c[f][j] : 0)) UT[j][p], i.e.
// (I - U U^T) w + U a with c = U^T w given (assembly of a full parameter from reduced
// coordinates and an unprojected complement), or w - U a with a = U^T w and c null
// (sign = -1: the complement of a whitened vector).
__global__ void dense_combine_kernel(int nf, int d_m, int r, double sign, const double* __restrict__ w,
                                     const double* __restrict__ a, const double* __restrict__ c,
                                     const double* __restrict__ UT, double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d_m) return;
    for (int f = blockIdx.y; f < nf; f += gridDim.y) {
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += (a[(long)f * r + j] - (c ? c[(long)f * r + j] : 0.0)) * UT[(long)j * d_m + p];
        out[(long)f * d_m + p] = (w ? w[(long)f * d_m + p] : 0.0) + sign * acc;
    }
}

// All d_m whitened coordinates (KLE order) of nf fields: the KLE gather with no reduced part.
static void whiten_full(const Basis& b, int nf, const double* fields, double* z, double* t1, double* t2,
                        hipStream_t st) {
    const int n = b.n;
    const dim3 grid((n * n + 255) / 256, grid_y(nf));
    // m[f][j][i] -> t1[f][k1][j] -> t2[f][k2][k1]
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, fields, b.q, 0, t1);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t1, b.q, 0, t2);
    hipLaunchKernelGGL(kle_gather_kernel, grid, dim3(256), 0, st, nf, n, 0, t2, b.perm, b.sqlam, (double*)nullptr, z);
}

// Nodal fields from all d_m whitened coordinates (z may alias fields).
static void unwhiten_full(const Basis& b, int nf, const double* z, double* fields, double* t1, double* t2,
                          hipStream_t st) {
    const int n = b.n;
    const dim3 grid((n * n + 255) / 256, grid_y(nf));
    // z -> t1[f][k2][k1] -> t2[f][i][k2] -> m[f][j][i]
    hipLaunchKernelGGL(kle_scatter_kernel, grid, dim3(256), 0, st, nf, n, 0, (const double*)nullptr, z, b.perm,
                       b.sqlam, t1);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t1, b.q, 1, t2);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t2, b.q, 1, fields);
}

void launch_encode(const Basis& b, int nf, const double* fields, double* x, double* zp, double* t1, double* t2,
                   hipStream_t st) {
    const int n = b.n;
    const dim3 grid((n * n + 255) / 256, grid_y(nf));
    if (b.dense) {
        // z = whitened coordinates (into t1); x = U^T z; z_perp = z - U x
        whiten_full(b, nf, fields, t1, t1, t2, st);
        double* xr = x ? x : t2;  // t2 is free once z is formed
        launch_gemm_nt64(nf, b.d_m, b.r, t1, b.d_m, b.UT, xr, b.r, nullptr, st);
        if (zp)
            hipLaunchKernelGGL(dense_combine_kernel, grid, dim3(256), 0, st, nf, b.d_m, b.r, -1.0, t1, xr,
                               (const double*)nullptr, b.UT, zp);
        DINO_HIP(hipGetLastError());
        return;
    }
    // m[f][j][i] -> t1[f][k1][j] -> t2[f][k2][k1]
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, fields, b.q, 0, t1);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t1, b.q, 0, t2);
    hipLaunchKernelGGL(kle_gather_kernel, grid, dim3(256), 0, st, nf, n, b.r, t2, b.perm, b.sqlam, x, zp);
    DINO_HIP(hipGetLastError());
}

void launch_decode(const Basis& b, int nf, const double* x, const double* zp, double* fields, double* t1, double* t2,
                   hipStream_t st) {
    const int n = b.n;
    const dim3 grid((n * n + 255) / 256, grid_y(nf));
    if (b.dense) {
        // z = U x + (I - U U^T) z_perp (into fields), then the nodal transform in place
        if (zp) launch_gemm_nt64(nf, b.d_m, b.r, zp, b.d_m, b.UT, t2, b.r, nullptr, st);
        hipLaunchKernelGGL(dense_combine_kernel, grid, dim3(256), 0, st, nf, b.d_m, b.r, 1.0, zp, x,
                           zp ? (const double*)t2 : nullptr, b.UT, fields);
        unwhiten_full(b, nf, fields, fields, t1, t2, st);
        DINO_HIP(hipGetLastError());
        return;
    }
    // z -> t1[f][k2][k1] -> t2[f][i][k2] -> m[f][j][i]
    hipLaunchKernelGGL(kle_scatter_kernel, grid, dim3(256), 0, st, nf, n, b.r, x, zp, b.perm, b.sqlam, t1);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t1, b.q, 1, t2);
    hipLaunchKernelGGL(sep_axis_kernel, grid, dim3(256), 0, st, nf, n, t2, b.q, 1, fields);
    DINO_HIP(hipGetLastError());
}

// dec[p][j] = F[j][p] (transpose of r x d_m rows)
__global__ void transpose_kernel(int rows, int cols, const double* __restrict__ F, double* __restrict__ D) {
    const long total = (long)rows * cols;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long p = e / rows;
        const int j = (int)(e % rows);
        D[e] = F[(long)j * cols + p];
    }
}

// var_perp[p] = prior variance[p] - sum_j dec[p][j]^2
__global__ void dense_var_perp_kernel(int d_m, int r, const double* __restrict__ pv, const double* __restrict__ dec,
                                      double* __restrict__ vp) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d_m) return;
    double s = 0.0;
    for (int j = 0; j < r; ++j) s += dec[(long)p * r + j] * dec[(long)p * r + j];
    vp[p] = pv[p] - s;
}

__global__ void to_float_rows_kernel(long total, const double* __restrict__ a, float* __restrict__ b) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
        b[e] = (float)a[e];
}

// A dense basis on the grid of b (its KLE order, q, perm and sqlam are kept): U (d_m x r,
// row-major, host) and optional DIS eigenvalues. Replaces dec, var_perp and lam_dev.
void build_dense_basis_device(Basis& b, const std::vector<double>& U, const double* lam_dis) {
    const int n = b.n, r = b.r, d_m = n * n;
    std::vector<double> ut((size_t)r * d_m);
    for (int p = 0; p < d_m; ++p)
        for (int j = 0; j < r; ++j) ut[(size_t)j * d_m + p] = U[(size_t)p * r + j];
    DINO_HIP(hipMalloc(&b.UT, sizeof(double) * ut.size()));
    DINO_HIP(hipMemcpy(b.UT, ut.data(), sizeof(double) * ut.size(), hipMemcpyHostToDevice));
    DINO_HIP(hipMalloc(&b.UT32, sizeof(float) * ut.size()));
    const long total = (long)r * d_m;
    const int gb = (int)std::min<long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(to_float_rows_kernel, dim3(gb), dim3(256), 0, 0, total, b.UT, b.UT32);
    b.lam_dis_host.clear();
    if (lam_dis) {
        b.lam_dis_host.assign(lam_dis, lam_dis + r);
        DINO_HIP(hipMalloc(&b.lam_dis, sizeof(double) * r));
        DINO_HIP(hipMemcpy(b.lam_dis, lam_dis, sizeof(double) * r, hipMemcpyHostToDevice));
    }
    // Psi_r = Q Lambda^1/2 U: the nodal fields of the basis vectors, transposed into dec
    double *F = nullptr, *t1 = nullptr, *t2 = nullptr, *Q2 = nullptr, *lamc = nullptr, *T = nullptr, *pv = nullptr;
    DINO_HIP(hipMalloc(&F, sizeof(double) * total));
    DINO_HIP(hipMalloc(&t1, sizeof(double) * total));
    DINO_HIP(hipMalloc(&t2, sizeof(double) * total));
    unwhiten_full(b, r, b.UT, F, t1, t2, 0);
    DINO_HIP(hipMalloc(&b.dec, sizeof(double) * total));
    hipLaunchKernelGGL(transpose_kernel, dim3(gb), dim3(256), 0, 0, r, d_m, F, b.dec);
    // prior pointwise variance (every mode), then the complement variance
    {
        const double h = 1.0 / (n - 1);
        std::vector<double> mu(n), lg((size_t)d_m);
        for (int k = 0; k < n; ++k) {
            const double sn = std::sin(M_PI * k / (2.0 * n));
            mu[k] = 4.0 * sn * sn;
        }
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                const double sm = mu[std::min(a, c)] + mu[std::max(a, c)];
                const double av = b.gamma * sm / (h * h) + b.delta;
                lg[(size_t)a * n + c] = 1.0 / (av * av);
            }
        DINO_HIP(hipMalloc(&lamc, sizeof(double) * d_m));
        DINO_HIP(hipMemcpy(lamc, lg.data(), sizeof(double) * d_m, hipMemcpyHostToDevice));
    }
    DINO_HIP(hipMalloc(&Q2, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&T, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&pv, sizeof(double) * d_m));
    const int g = (d_m + 255) / 256;
    hipLaunchKernelGGL(q2_kernel, dim3(g), dim3(256), 0, 0, n, Q2);
    hipLaunchKernelGGL(vp_stage1_kernel, dim3(g), dim3(256), 0, 0, n, Q2, lamc, T);
    hipLaunchKernelGGL(vp_stage2_kernel, dim3(g), dim3(256), 0, 0, n, Q2, T, pv);
    DINO_HIP(hipMalloc(&b.var_perp, sizeof(double) * d_m));
    hipLaunchKernelGGL(dense_var_perp_kernel, dim3(g), dim3(256), 0, 0, d_m, r, pv, b.dec, b.var_perp);
    DINO_HIP(hipGetLastError());
    DINO_HIP(hipDeviceSynchronize());
    hipFree(F);
    hipFree(t1);
    hipFree(t2);
    hipFree(Q2);
    hipFree(lamc);
    hipFree(T);
    hipFree(pv);
    b.dense = true;
}

void build_basis_device(Basis& b) {
    const int n = b.n, r = b.r, d_m = n * n;
    int32_t *k1d = nullptr, *k2d = nullptr;
    double *Q2 = nullptr, *lamc = nullptr, *T = nullptr;
    DINO_HIP(hipMalloc(&b.dec, sizeof(double) * (size_t)d_m * r));
    DINO_HIP(hipMalloc(&b.var_perp, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&b.lam_dev, sizeof(double) * r));
    DINO_HIP(hipMalloc(&k1d, sizeof(int32_t) * r));
    DINO_HIP(hipMalloc(&k2d, sizeof(int32_t) * r));
    DINO_HIP(hipMalloc(&Q2, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&lamc, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&T, sizeof(double) * d_m));
    DINO_HIP(hipMemcpy(k1d, b.k1.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(k2d, b.k2.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(b.lam_dev, b.lam.data(), sizeof(double) * r, hipMemcpyHostToDevice));
    // complement eigenvalue grid lamc[k1][k2] (kept modes zeroed), from the host ordering
    {
        const double h = 1.0 / (n - 1);
        std::vector<double> mu(n), lg((size_t)d_m);
        for (int k = 0; k < n; ++k) {
            const double sn = std::sin(M_PI * k / (2.0 * n));
            mu[k] = 4.0 * sn * sn;
        }
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                const double s = mu[std::min(a, c)] + mu[std::max(a, c)];
                const double av = b.gamma * s / (h * h) + b.delta;
                lg[(size_t)a * n + c] = 1.0 / (av * av);
            }
        for (int j = 0; j < r; ++j) lg[(size_t)b.k1[j] * n + b.k2[j]] = 0.0;
        DINO_HIP(hipMemcpy(lamc, lg.data(), sizeof(double) * d_m, hipMemcpyHostToDevice));
    }
    const long total = (long)d_m * r;
    hipLaunchKernelGGL(basis_dec_kernel, dim3((int)std::min<long>((total + 255) / 256, 16384)), dim3(256), 0, 0, n,
                       r, k1d, k2d, b.lam_dev, b.dec);
    const int g = (d_m + 255) / 256;
    hipLaunchKernelGGL(q2_kernel, dim3(g), dim3(256), 0, 0, n, Q2);
    hipLaunchKernelGGL(vp_stage1_kernel, dim3(g), dim3(256), 0, 0, n, Q2, lamc, T);
    hipLaunchKernelGGL(vp_stage2_kernel, dim3(g), dim3(256), 0, 0, n, Q2, T, b.var_perp);
    // full KLE order (mode of every position) and sqrt(lambda) for encode / decode
    DINO_HIP(hipMalloc(&b.q, sizeof(double) * d_m));
    DINO_HIP(hipMalloc(&b.perm, sizeof(int32_t) * d_m));
    DINO_HIP(hipMalloc(&b.sqlam, sizeof(double) * d_m));
    hipLaunchKernelGGL(q_kernel, dim3(g), dim3(256), 0, 0, n, b.q);
    DINO_HIP(hipMemcpy(b.perm, b.order.data(), sizeof(int32_t) * d_m, hipMemcpyHostToDevice));
    DINO_HIP(hipMemcpy(b.sqlam, b.sqlam_all.data(), sizeof(double) * d_m, hipMemcpyHostToDevice));
    DINO_HIP(hipGetLastError());
    DINO_HIP(hipDeviceSynchronize());
    hipFree(k1d);
    hipFree(k2d);
    hipFree(Q2);
    hipFree(lamc);
    hipFree(T);
}

// ---------------------------------------------------------------------------------
// Posterior moments from the trace rows [b, N): xbar (r), S (r x r, divide by count).
__global__ void trace_mean_kernel(long nsamp, int r, const float* __restrict__ X, double* __restrict__ xbar) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (long s = threadIdx.x; s < nsamp; s += blockDim.x) acc += (double)X[s * r + j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) xbar[j] = red[0] / (double)nsamp;
}

__global__ __launch_bounds__(256) void trace_cov_kernel(long nsamp, int r, const float* __restrict__ X,
                                                        const double* __restrict__ xbar, double* __restrict__ S) {
    __shared__ double Aj[32][33];
    __shared__ double Ak[32][33];
    const int j0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (long s0 = 0; s0 < nsamp; s0 += 32) {
        for (int e = tid; e < 32 * 32; e += 256) {
            const int ss = e >> 5, jj = e & 31;
            const long s = s0 + ss;
            Aj[ss][jj] = (s < nsamp && j0 + jj < r) ? (double)X[s * r + j0 + jj] - xbar[j0 + jj] : 0.0;
            Ak[ss][jj] = (s < nsamp && k0 + jj < r) ? (double)X[s * r + k0 + jj] - xbar[k0 + jj] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int ss = 0; ss < 32; ++ss) {
            const double a0 = Aj[ss][ty], a1 = Aj[ss][ty + 16], b0 = Ak[ss][tx], b1 = Ak[ss][tx + 16];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + ty + 16 * a, k = k0 + tx + 16 * b;
            if (j < r && k < r) S[(long)j * r + k] = acc[a][b] / (double)nsamp;
        }
}

// mean_p = sum_j dec[p][j] xbar_j ; var_p = dec[p] S dec[p]^T + var_perp[p]
__global__ void field_moments_kernel(int d_m, int r, const double* __restrict__ dec, const double* __restrict__ xbar,
                                     const double* __restrict__ S, const double* __restrict__ vp,
                                     double* __restrict__ mean, double* __restrict__ var) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d_m) return;
    const double* dp = dec + (long)p * r;
    double m = 0.0, v = 0.0;
    for (int j = 0; j < r; ++j) {
        m += dp[j] * xbar[j];
        double t = 0.0;
        for (int k = 0; k < r; ++k) t += S[(long)j * r + k] * dp[k];
        v += dp[j] * t;
    }
    mean[p] = m;
    var[p] = v + vp[p];
}

void launch_posterior(dino_problem* p, int burn_in, double* mean, double* var, double* xbar, double* S,
                      hipStream_t st) {
    const long rows = p->recorded - burn_in;
    const long nsamp = rows * p->C;
    const float* X = p->xtrace + (long)burn_in * p->C * p->r;
    const int r = p->r;
    hipLaunchKernelGGL(trace_mean_kernel, dim3(r), dim3(256), 0, st, nsamp, r, X, xbar);
    const int t = (r + 31) / 32;
    hipLaunchKernelGGL(trace_cov_kernel, dim3(t, t), dim3(256), 0, st, nsamp, r, X, xbar, S);
    const Basis& b = p->ctx->basis;
    hipLaunchKernelGGL(field_moments_kernel, dim3((b.d_m + 127) / 128), dim3(128), 0, st, b.d_m, r, b.dec, xbar, S,
                       b.var_perp, mean, var);
    DINO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------
// ESS fraction per coordinate (eq. ess reading). Y[j][c][i] holds centred samples
// (chain means removed); one block per coordinate walks the lags in pairs.
__global__ void ess_center_kernel(int n, int C, int r, const float* __restrict__ X, double* __restrict__ Y,
                                  double* __restrict__ cmean) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    for (int c = blockIdx.y; c < C; c += gridDim.y) {  // the grid's y extent is capped at GRID_Y_MAX
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)X[((long)i * C + c) * r + j];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        const double m = red[0] / n;
        if (threadIdx.x == 0) cmean[(long)j * C + c] = m;
        double* y = Y + ((long)j * C + c) * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = (double)X[((long)i * C + c) * r + j] - m;
        __syncthreads();  // red is rewritten for the next chain
    }
}

__device__ double block_reduce_256(double v, double* red) {
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// sum over chains of the biased lag-t autocovariance numerators: sum_c sum_i y_ci y_c(i+t)
__device__ double lag_sum(const double* y, int C, int n, int t, double* red) {
    double acc = 0.0;
    const long m = n - t;
    for (long e = threadIdx.x; e < (long)C * m; e += blockDim.x) {
        const long c = e / m, i = e % m;
        acc += y[c * n + i] * y[c * n + i + t];
    }
    return block_reduce_256(acc, red);
}

__global__ void ess_kernel(int n, int C, const double* __restrict__ Y, const double* __restrict__ cmean,
                           double* __restrict__ ess) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const double* y = Y + (long)j * C * n;
    // w: mean within-chain variance (divide by n - 1); v: pooled variance
    const double ss = lag_sum(y, C, n, 0, red);
    const double w = ss / ((double)C * (n - 1));
    double gm = 0.0;
    for (int c = 0; c < C; ++c) gm += cmean[(long)j * C + c];
    gm /= C;
    double bsum = 0.0;
    for (int c = 0; c < C; ++c) {
        const double d = cmean[(long)j * C + c] - gm;
        bsum += d * d;
    }
    double v = (double)(n - 1) / n * w;
    if (C > 1) v += (double)(C + 1) / ((double)C * (C - 1)) * bsum;
    if (!(v > 0.0)) {
        if (threadIdx.x == 0) ess[j] = NAN;
        return;
    }
    auto rho = [&](int t) {
        const double ac = lag_sum(y, C, n, t, red) / ((double)n * C);
        return 1.0 - (w - ac) / v;
    };
    double total = 0.0;
    for (int tp = 0; 2 * tp + 1 < n; ++tp) {
        const double re = (tp == 0) ? 1.0 : rho(2 * tp);
        const double ro = rho(2 * tp + 1);
        if (re + ro <= 0.0) break;
        total += (tp > 0 ? re : 0.0) + ro;
    }
    if (threadIdx.x == 0) ess[j] = 1.0 / (1.0 + 2.0 * total);
}

void launch_ess(dino_problem* p, int burn_in, double* ess, hipStream_t st) {
    const int n = (int)(p->recorded - burn_in), C = p->C, r = p->r;
    double *Y = nullptr, *cm = nullptr;
    DINO_HIP(hipMalloc(&Y, sizeof(double) * (size_t)r * C * n));
    DINO_HIP(hipMalloc(&cm, sizeof(double) * (size_t)r * C));
    const float* X = p->xtrace + (long)burn_in * C * r;
    hipLaunchKernelGGL(ess_center_kernel, dim3(r, grid_y(C)), dim3(256), 0, st, n, C, r, X, Y, cm);
    hipLaunchKernelGGL(ess_kernel, dim3(r), dim3(256), 0, st, n, C, Y, cm, ess);
    DINO_HIP(hipGetLastError());
    DINO_HIP(hipStreamSynchronize(st));
    hipFree(Y);
    hipFree(cm);
}

}  // namespace dino
