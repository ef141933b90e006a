// Learned per-leaf block preconditioner: a 3-layer MLP (ReLU) with BF16
// inference weights and FP32 accumulation, trained on the device with Adam
// (FP32 master weights).  Hand-written kernels: feature extraction from a
// residual, tiled FP32 GEMM (forward and backward), masked MSE loss, Adam.
//
// Rows are chunks of <= 64 consecutive elements of one leaf L of the plan's
// tree (a single row per leaf when n_L <= 64).  For a residual v and a row R
// of leaf L:
//   z_R  = rows R of the block-Jacobi correction inv(A_LL) v_L
//   s_R  = |v_R| times the unit phase of the row's largest entry of v
//   features (272): Re, Im of v_R / s_R and of z_R / s_R (each zero-padded
//                   to 64), leaf width in wavelengths, the mesh's largest
//                   edge in wavelengths, n_R / 64, 1, 0...
//   output (128):   Re / Im of a 64-element correction c_R
//   preconditioner: M(v)_R = z_R + s_R c_R  (so M(a v) = a M(v), a complex)
// Training target for a pair (r, e = A^-1 r): (e_R - z_R) / s_R, masked to
// the row's n_R elements.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "mlp.hpp"

namespace fda {

// ------------------------------------------------------------------ BF16

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
    uint32_t r = ((u >> 16) & 1u) + 0x7fffu;  // round to nearest even
    return (uint16_t)((u + r) >> 16);
}

__global__ void k_to_bf16(const float *in, uint16_t *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f32_to_bf16(in[i]);
}

// ------------------------------------------------------------------ GEMM
// C[M x N] = act(op(A) op(B) + bias), FP32 accumulation.  op(A) is M x K,
// op(B) is K x N; row-major storage with leading dimensions lda, ldb, ldc;
// transA: A is stored K x M; transB: B is stored N x K.  B may be BF16.
// 64 x 64 tiles, 256 threads, 4 x 4 outputs per thread.
template <class TB>
__device__ __forceinline__ float ldB(const TB *B, int64_t i);
template <>
__device__ __forceinline__ float ldB<float>(const float *B, int64_t i) { return B[i]; }
template <>
__device__ __forceinline__ float ldB<uint16_t>(const uint16_t *B, int64_t i) { return bf16_to_f32(B[i]); }

template <class TB>
__global__ void __launch_bounds__(256) k_gemm_f32(int M, int N, int K, const float *A, int lda, int transA,
                                                  const TB *B, int ldb, int transB, float *C, int ldc,
                                                  const float *bias, int relu, int accumulate) {
    __shared__ float As[16][64 + 1];
    __shared__ float Bs[16][64 + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int gm = m0 + mm, gk = k0 + kk;
            float a = 0.f;
            if (gm < M && gk < K) a = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[kk][mm] = a;
            const int gn = n0 + mm;
            float b = 0.f;
            if (gn < N && gk < K) b = transB ? ldB<TB>(B, (int64_t)gn * ldb + gk) : ldB<TB>(B, (int64_t)gk * ldb + gn);
            Bs[kk][mm] = b;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty + 16 * i;
        if (gm >= M) continue;
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx + 16 * j;
            if (gn >= N) continue;
            float v = acc[i][j] + (bias ? bias[gn] : 0.f);
            if (relu) v = fmaxf(v, 0.f);
            float *c = C + (int64_t)gm * ldc + gn;
            *c = accumulate ? *c + v : v;
        }
    }
}

template <class TB>
static void gemm(int M, int N, int K, const float *A, int lda, int transA, const TB *B, int ldb, int transB, float *C,
                 int ldc, const float *bias, int relu, int accumulate, hipStream_t st) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL(k_gemm_f32<TB>, grid, dim3(256), 0, st, M, N, K, A, lda, transA, B, ldb, transB, C, ldc, bias,
                       relu, accumulate);
}

// Forward-pass product on the matrix cores: C[M x N] = act(bf16(A) W + bias)
// with v_mfma_f32_16x16x16bf16_1k (BF16 operands, FP32 accumulation).  The
// FP32 activations A (row-major, lda) are rounded to bfloat16 as they are
// loaded; W is the BF16 weight copy (row-major K x N, ldw).  A workgroup of
// four waves computes a 64 x 64 tile: wave w rows 16 w .. 16 w + 15, four
// 16-column tiles.  Operand layout per lane l: A row l % 16 and B column
// l % 16, k-slots 4 (l / 16) .. 4 (l / 16) + 3; result column l % 16, rows
// 4 (l / 16) .. + 3.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float *A, int lda, const uint16_t *W,
                                                   int ldw, float *C, int ldc, const float *bias, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int m0 = blockIdx.y * 64 + wave * 16, n0 = blockIdx.x * 64;
    const int arow = m0 + li;
    f32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 4 * lk + j;
            const float v = (arow < M && k < K) ? A[(int64_t)arow * lda + k] : 0.f;
            a[j] = (short)f32_to_bf16(v);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = n0 + 16 * c + li;
            bf16x4 b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + 4 * lk + j;
                b[j] = (short)((k < K && n < N) ? W[(int64_t)k * ldw + n] : 0);
            }
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = n0 + 16 * c + li;
        if (n >= N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = m0 + 4 * lk + v;
            if (r >= M) continue;
            float o = acc[c][v] + (bias ? bias[n] : 0.f);
            if (relu) o = fmaxf(o, 0.f);
            C[(int64_t)r * ldc + n] = o;
        }
    }
}

static void gemm_bf16(int M, int N, int K, const float *A, int lda, const uint16_t *W, int ldw, float *C, int ldc,
                      const float *bias, int relu, hipStream_t st) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, M, N, K, A, lda, W, ldw, C, ldc, bias, relu);
}

// ------------------------------------------------------------------ training pieces

// dY = 2 mask (Y - T) / count; partial sums of mask (Y - T)^2 per block.
__global__ void k_mse_grad(const float *Y, const float *T, const float *Mk, int64_t n, float inv_count, float *dY,
                           float *partial) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = Mk[i] * (Y[i] - T[i]);
        dY[i] = 2.f * d * inv_count;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dH *= (H > 0)
__global__ void k_relu_back(const float *H, float *dH, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (H[i] <= 0.f) dH[i] = 0.f;
}

// db[j] = sum_i dY[i, j]
__global__ void k_colsum(const float *dY, int M, int N, float *db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += dY[(int64_t)i * N + j];
    db[j] = s;
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// rows of X, T, Mask selected by idx
__global__ void k_gather_rows(const float *src, int width, const int32_t *idx, int rows, float *dst) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rows * width;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / width), c = (int)(e % width);
        dst[e] = src[(int64_t)idx[r] * width + c];
    }
}

// ------------------------------------------------------------------ features

// Complex helpers for the row scale s (|s| = |v_R|, arg s = phase of the
// row's largest entry): features and outputs live in the frame v / s, so the
// preconditioner satisfies M(a v) = a M(v) for every complex a.
__device__ __forceinline__ double2 cdiv_scale(double2 x, double2 s) {
    const double d = s.x * s.x + s.y * s.y;
    if (d == 0.0) return make_double2(0.0, 0.0);
    return make_double2((x.x * s.x + x.y * s.y) / d, (x.y * s.x - x.x * s.y) / d);
}

// One block of 64 threads per row (a chunk of <= 64 consecutive elements of
// one leaf); v in tree order (one column).  The block-Jacobi correction of
// the row's elements uses the whole leaf: z_i = sum_j inv(A_LL)[i, j] v_j.
// Writes the row's features, its scale s and z on the row's elements.
__global__ void k_mlp_features(const int64_t *leaf_off, const int64_t *row_off, const int32_t *row_leaf,
                               const int32_t *row_n, const int64_t *inv_off, const double2 *inv, const double2 *v,
                               const float *leaf_scalars, float *feat, double2 *rscale, double2 *z) {
    extern __shared__ double2 vleaf[];  // the leaf's v (max_leaf entries)
    __shared__ double red[64];
    __shared__ double bmag[64];
    __shared__ int bidx[64];
    const int row = blockIdx.x, t = threadIdx.x;
    const int b = row_leaf[row];
    const int64_t l0 = leaf_off[b];
    const int nL = (int)(leaf_off[b + 1] - l0);
    const int64_t e0 = row_off[row];
    const int n = row_n[row];
    const int i0 = (int)(e0 - l0);  // row offset inside the leaf
    for (int j = t; j < nL; j += 64) vleaf[j] = v[l0 + j];
    __syncthreads();
    double2 vi = make_double2(0.0, 0.0);
    if (t < n) vi = vleaf[i0 + t];
    const double m2 = vi.x * vi.x + vi.y * vi.y;
    red[t] = m2;
    bmag[t] = m2;
    bidx[t] = t;
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) {
        if (t < o) {
            red[t] += red[t + o];
            // largest modulus, ties to the smaller index
            if (bmag[t + o] > bmag[t] || (bmag[t + o] == bmag[t] && bidx[t + o] < bidx[t])) {
                bmag[t] = bmag[t + o];
                bidx[t] = bidx[t + o];
            }
        }
        __syncthreads();
    }
    const double nv = sqrt(red[0]);
    double2 s = make_double2(0.0, 0.0);
    if (nv > 0) {
        const double2 vm = vleaf[i0 + bidx[0]];
        const double am = sqrt(bmag[0]);
        s = make_double2(nv * vm.x / am, nv * vm.y / am);
    }
    double2 zi = make_double2(0.0, 0.0);
    if (t < n) {
        const double2 *A = inv + inv_off[b];
        const int i = i0 + t;
        for (int j = 0; j < nL; ++j) {
            const double2 a = A[i + (int64_t)j * nL], x = vleaf[j];
            zi.x += a.x * x.x - a.y * x.y;
            zi.y += a.x * x.y + a.y * x.x;
        }
        z[e0 + t] = zi;
    }
    const double2 vt = cdiv_scale(vi, s), zt = cdiv_scale(zi, s);
    float *f = feat + (int64_t)row * kMlpIn;
    f[t] = (float)vt.x;
    f[64 + t] = (float)vt.y;
    f[128 + t] = (float)zt.x;
    f[192 + t] = (float)zt.y;
    if (t < kMlpIn - 256) {
        float sc = 0.f;
        if (t < 2) sc = leaf_scalars[2 * b + t];
        else if (t == 2) sc = n / 64.f;
        else if (t == 3) sc = 1.f;
        f[256 + t] = sc;
    }
    if (t == 0) rscale[row] = s;
}

// out_row = z_row + s_row c_row (tree order); flags non-finite outputs.
__global__ void k_mlp_apply(const int64_t *row_off, const int32_t *row_n, const float *Y, const double2 *rscale,
                            const double2 *z, double2 *out, int *bad) {
    const int row = blockIdx.x, t = threadIdx.x;
    const int64_t e0 = row_off[row];
    const int n = row_n[row];
    if (t >= n) return;
    const float cr = Y[(int64_t)row * kMlpOut + t], ci = Y[(int64_t)row * kMlpOut + 64 + t];
    if (!isfinite(cr) || !isfinite(ci)) {
        *bad = 1;
        out[e0 + t] = z[e0 + t];
        return;
    }
    const double2 s = rscale[row];
    const double2 zz = z[e0 + t];
    out[e0 + t] = make_double2(zz.x + s.x * cr - s.y * ci, zz.y + s.x * ci + s.y * cr);
}

// Training targets: (e_row - z_row) / s_row and the mask of the row's elements.
__global__ void k_mlp_targets(const int64_t *row_off, const int32_t *row_n, const double2 *e, const double2 *z,
                              const double2 *rscale, float *tgt, float *mask) {
    const int row = blockIdx.x, t = threadIdx.x;
    const int64_t e0 = row_off[row];
    const int n = row_n[row];
    const double2 s = rscale[row];
    float tr = 0.f, ti = 0.f, mk = 0.f;
    if (t < n) {
        const double2 ee = e[e0 + t], zz = z[e0 + t];
        const double2 d = cdiv_scale(make_double2(ee.x - zz.x, ee.y - zz.y), s);
        tr = (float)d.x;
        ti = (float)d.y;
        mk = 1.f;
    }
    tgt[(int64_t)row * kMlpOut + t] = tr;
    tgt[(int64_t)row * kMlpOut + 64 + t] = ti;
    mask[(int64_t)row * kMlpOut + t] = mk;
    mask[(int64_t)row * kMlpOut + 64 + t] = mk;
}

// ------------------------------------------------------------------ model

static size_t param_count(int h) { return (size_t)kMlpIn * h + h + (size_t)h * h + h + (size_t)h * kMlpOut + kMlpOut; }

void Mlp::offsets(size_t &w1, size_t &b1, size_t &w2, size_t &b2, size_t &w3, size_t &b3) const {
    w1 = 0;
    b1 = w1 + (size_t)kMlpIn * hidden;
    w2 = b1 + hidden;
    b2 = w2 + (size_t)hidden * hidden;
    w3 = b2 + hidden;
    b3 = w3 + (size_t)hidden * kMlpOut;
}

static void chk(hipError_t e, const char *w) {
    if (e != hipSuccess) throw MlpError{std::string(w) + ": " + hipGetErrorString(e)};
}

Mlp *mlp_create(int hidden, uint64_t seed) {
    Mlp *m = new Mlp();
    m->hidden = hidden;
    m->nparam = param_count(hidden);
    size_t w1, b1, w2, b2, w3, b3;
    m->offsets(w1, b1, w2, b2, w3, b3);
    // He-normal init of the weights, zero biases
    std::vector<float> p(m->nparam, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](size_t off, int fan_in, size_t count) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / fan_in));
        for (size_t i = 0; i < count; ++i) p[off + i] = nd(rng);
    };
    fill(w1, kMlpIn, (size_t)kMlpIn * hidden);
    fill(w2, hidden, (size_t)hidden * hidden);
    fill(w3, hidden, (size_t)hidden * kMlpOut);
    for (size_t i = 0; i < (size_t)hidden * kMlpOut; ++i) p[w3 + i] *= 0.1f;  // start near block-Jacobi
    chk(hipMalloc(&m->w, sizeof(float) * m->nparam), "alloc");
    chk(hipMalloc(&m->wb, sizeof(uint16_t) * m->nparam), "alloc");
    chk(hipMemcpy(m->w, p.data(), sizeof(float) * m->nparam, hipMemcpyHostToDevice), "h2d");
    m->sync_bf16(nullptr);
    return m;
}

void Mlp::sync_bf16(hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(256), dim3(256), 0, st, w, wb, (int64_t)nparam);
}

void mlp_free(Mlp *m) {
    if (!m) return;
    hipFree(m->w);
    hipFree(m->wb);
    for (void *q : m->work) hipFree(q);
    delete m;
}

void Mlp::ensure_rows(int64_t rows) {
    if (rows <= cap_rows) return;
    for (void *q : work) hipFree(q);
    work.clear();
    auto al = [&](size_t n) {
        void *q = nullptr;
        chk(hipMalloc(&q, std::max<size_t>(n, 4) * sizeof(float)), "alloc");
        work.push_back(q);
        return (float *)q;
    };
    h1 = al((size_t)rows * hidden);
    h2 = al((size_t)rows * hidden);
    cap_rows = rows;
}

// Y (rows x 128) = MLP(X (rows x 272)): each layer a BF16 product on the
// matrix cores (layer input and weights in bfloat16, FP32 accumulation,
// bias and ReLU in FP32); the hidden activations go to a1 and a2 (rows x
// hidden floats each, before rounding).
void Mlp::forward_into(const float *X, int64_t rows, float *Y, float *a1, float *a2, hipStream_t st) const {
    size_t w1, b1, w2, b2, w3, b3;
    offsets(w1, b1, w2, b2, w3, b3);
    gemm_bf16((int)rows, hidden, kMlpIn, X, kMlpIn, wb + w1, hidden, a1, hidden, w + b1, 1, st);
    gemm_bf16((int)rows, hidden, hidden, a1, hidden, wb + w2, hidden, a2, hidden, w + b2, 1, st);
    gemm_bf16((int)rows, kMlpOut, hidden, a2, hidden, wb + w3, kMlpOut, Y, kMlpOut, w + b3, 0, st);
}

void Mlp::forward(const float *X, int64_t rows, float *Y, hipStream_t st) {
    ensure_rows(rows);
    forward_into(X, rows, Y, h1, h2, st);
}

// ------------------------------------------------------------------ allocation-free forward pass
// For callers that cannot allocate device memory: the hidden activations
// live in one statically allocated array per device, so the pass needs no
// hipMalloc.  Every call on a device shares its array (concurrent calls on
// one device race); it is never cleared, since the first layer overwrites
// every activation it later reads.
static __device__ __align__(256) float scratch[kMlpNoAllocFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device ordinal
}  // namespace

int64_t mlp_noalloc_max_rows(int hidden) { return kMlpNoAllocFloats / (2 * (int64_t)hidden); }

// Device address of `scratch` on `device`, which must be the current device;
// looked up once per device (the array's name is only a host-side stand-in).
static float *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) throw MlpError{"device ordinal out of range for the static scratch"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        chk(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) throw MlpError{"hipGetSymbolAddress(scratch) returned a null address"};
        g_scratch_dev[device] = (float *)ptr;
    }
    return g_scratch_dev[device];
}

void Mlp::forward_noalloc(const float *X, int64_t rows, float *Y, int device, hipStream_t st) const {
    if (rows > mlp_noalloc_max_rows(hidden)) throw MlpError{"rows exceed the static scratch"};
    float *ws = noalloc_scratch(device);
    forward_into(X, rows, Y, ws, ws + rows * (int64_t)hidden, st);
}

// Gradient of the masked MSE (mean over rows x 128 outputs) of one batch
// with respect to every parameter, written to g (nparam floats); returns the
// sum of squared masked errors.  The forward pass and the products with the
// weights use the BF16 copy (straight-through: the gradient is applied to the
// FP32 master).  Needs m->ensure_rows(rows) and the scratch of MlpGradWork.
double MlpGradWork::run(Mlp *m, const float *xb, const float *tb, const float *mb, int rows, float *g,
                        hipStream_t st) {
    const int h = m->hidden;
    size_t w1, b1, w2, b2, w3, b3;
    m->offsets(w1, b1, w2, b2, w3, b3);
    m->forward(xb, rows, yb, st);
    const float inv_count = 1.f / (float)((int64_t)rows * kMlpOut);
    hipLaunchKernelGGL(k_mse_grad, dim3(256), dim3(256), 0, st, yb, tb, mb, (int64_t)rows * kMlpOut, inv_count, dy,
                       part);
    gemm<float>(h, kMlpOut, rows, m->h2, h, 1, dy, kMlpOut, 0, g + w3, kMlpOut, nullptr, 0, 0, st);
    hipLaunchKernelGGL(k_colsum, dim3((kMlpOut + 127) / 128), dim3(128), 0, st, dy, rows, kMlpOut, g + b3);
    gemm<uint16_t>(rows, h, kMlpOut, dy, kMlpOut, 0, m->wb + w3, kMlpOut, 1, dh2, h, nullptr, 0, 0, st);
    hipLaunchKernelGGL(k_relu_back, dim3(256), dim3(256), 0, st, m->h2, dh2, (int64_t)rows * h);
    gemm<float>(h, h, rows, m->h1, h, 1, dh2, h, 0, g + w2, h, nullptr, 0, 0, st);
    hipLaunchKernelGGL(k_colsum, dim3((h + 127) / 128), dim3(128), 0, st, dh2, rows, h, g + b2);
    gemm<uint16_t>(rows, h, h, dh2, h, 0, m->wb + w2, h, 1, dh1, h, nullptr, 0, 0, st);
    hipLaunchKernelGGL(k_relu_back, dim3(256), dim3(256), 0, st, m->h1, dh1, (int64_t)rows * h);
    gemm<float>(kMlpIn, h, rows, xb, kMlpIn, 1, dh1, h, 0, g + w1, h, nullptr, 0, 0, st);
    hipLaunchKernelGGL(k_colsum, dim3((h + 127) / 128), dim3(128), 0, st, dh1, rows, h, g + b1);
    chk(hipGetLastError(), "gradient");
    std::vector<float> ph(256);
    chk(hipMemcpyAsync(ph.data(), part, sizeof(float) * 256, hipMemcpyDeviceToHost, st), "d2h");
    chk(hipStreamSynchronize(st), "sync");
    double s = 0;
    for (float v : ph) s += v;
    return s;
}

MlpGradWork::MlpGradWork(const Mlp *m, int batch) {
    const int h = m->hidden;
    yb = al((size_t)batch * kMlpOut);
    dy = al((size_t)batch * kMlpOut);
    dh2 = al((size_t)batch * h);
    dh1 = al((size_t)batch * h);
    part = al(256);
}

float *MlpGradWork::al(size_t count) {
    void *q = nullptr;
    chk(hipMalloc(&q, std::max<size_t>(count, 4) * sizeof(float)), "alloc");
    bufs.push_back(q);
    return (float *)q;
}

MlpGradWork::~MlpGradWork() {
    for (void *q : bufs) hipFree(q);
}

double mlp_gradient(Mlp *m, const float *X, const float *T, const float *Mk, int64_t n, float *g, hipStream_t st) {
    m->ensure_rows(n);
    MlpGradWork wk(m, (int)n);
    return wk.run(m, X, T, Mk, (int)n, g, st);
}

std::vector<double> mlp_train(Mlp *m, const float *X, const float *T, const float *Mk, int64_t n, int epochs,
                              int batch, float lr, uint64_t seed, hipStream_t st) {
    std::vector<void *> tmp;
    auto al = [&](size_t count) {
        void *q = nullptr;
        chk(hipMalloc(&q, std::max<size_t>(count, 4) * sizeof(float)), "alloc");
        tmp.push_back(q);
        return (float *)q;
    };
    std::vector<double> losses;
    try {
        float *g = al(m->nparam), *mo = al(m->nparam), *vo = al(m->nparam);
        chk(hipMemsetAsync(mo, 0, sizeof(float) * m->nparam, st), "zero");
        chk(hipMemsetAsync(vo, 0, sizeof(float) * m->nparam, st), "zero");
        float *xb = al((size_t)batch * kMlpIn), *tb = al((size_t)batch * kMlpOut), *mb = al((size_t)batch * kMlpOut);
        int32_t *idx_d = (int32_t *)al((size_t)std::max<int64_t>(n, 1));
        m->ensure_rows(batch);
        MlpGradWork wk(m, batch);
        std::vector<int32_t> idx(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
        std::mt19937_64 rng(seed);
        const float b1c = 0.9f, b2c = 0.999f, eps = 1e-8f;
        int64_t step = 0;
        for (int ep = 0; ep < epochs; ++ep) {
            std::shuffle(idx.begin(), idx.end(), rng);
            chk(hipMemcpyAsync(idx_d, idx.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st), "h2d");
            double loss_sum = 0, count = 0;
            for (int64_t r0 = 0; r0 < n; r0 += batch) {
                const int rows = (int)std::min<int64_t>(batch, n - r0);
                hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, st, X, kMlpIn, idx_d + r0, rows, xb);
                hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, st, T, kMlpOut, idx_d + r0, rows, tb);
                hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, st, Mk, kMlpOut, idx_d + r0, rows, mb);
                loss_sum += wk.run(m, xb, tb, mb, rows, g, st);
                count += (double)rows * kMlpOut;
                ++step;
                const float c1 = 1.f - std::pow(b1c, (float)step), c2 = 1.f - std::pow(b2c, (float)step);
                hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, st, m->w, g, mo, vo, (int64_t)m->nparam, lr, b1c,
                                   b2c, c1, c2, eps);
                m->sync_bf16(st);
                chk(hipGetLastError(), "train step");
            }
            losses.push_back(loss_sum / std::max(1.0, count));
        }
        chk(hipStreamSynchronize(st), "sync");
    } catch (...) {
        hipStreamSynchronize(st);
        for (void *q : tmp) hipFree(q);
        throw;
    }
    for (void *q : tmp) hipFree(q);
    return losses;
}

void mlp_features(const DevPlan &d, const double2 *vt, const float *leaf_scalars, float *feat, double2 *rscale,
                  double2 *z, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)d.mlp_nrows), dim3(64), sizeof(double2) * d.max_leaf, st,
                       d.leaf_off, d.mlp_row_off, d.mlp_row_leaf, d.mlp_row_n, d.bj_off, d.bj_inv, vt, leaf_scalars,
                       feat, rscale, z);
}

void mlp_apply(const DevPlan &d, const float *Y, const double2 *rscale, const double2 *z, double2 *out, int *bad,
               hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_apply, dim3((unsigned)d.mlp_nrows), dim3(64), 0, st, d.mlp_row_off, d.mlp_row_n, Y,
                       rscale, z, out, bad);
}

void mlp_targets(const DevPlan &d, const double2 *et, const double2 *z, const double2 *rscale, float *tgt,
                 float *mask, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)d.mlp_nrows), dim3(64), 0, st, d.mlp_row_off, d.mlp_row_n, et,
                       z, rscale, tgt, mask);
}

}  // namespace fda
