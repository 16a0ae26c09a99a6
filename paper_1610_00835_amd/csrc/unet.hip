// Learned right preconditioner: a three-level 3D convolutional U-Net (widths
// w1/w2/w3, 3x3x3 convolutions, 2x2x2 average pooling, nearest upsampling,
// skip connections by concatenation), trained on the device.
//
// Data layout: activations are FP32, channels-last ([batch][voxel][channel],
// voxel = x-fastest cell index of the solver grid), so one voxel's channels are
// contiguous and a 3x3x3 convolution is an implicit GEMM with a reduction over
// (tap, input channel).  Convolutions of the forward pass and the input
// gradients of the backward pass run on the matrix cores as BF16 x BF16 -> FP32
// (v_mfma_f32_16x16x32_bf16), BF16 weights times the FP32 activations split
// into two BF16 parts (hi + lo, two products, so activations keep ~16 mantissa
// bits and rounding noise does not compound layer after layer): rows are output
// channels, columns are voxels, so
// each lane ends with four consecutive channels of one voxel (one 16-byte
// store).  Weight gradients use FP32 operands (v_mfma_f32_16x16x4f32) with the
// voxel sum split into slabs and summed in a fixed order (deterministic).
// Parameters live in one flat FP32 vector in the canonical layout documented in
// include/ertvie.h; BF16 copies in GEMM order are rebuilt after every update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

namespace ertvie {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kNetLayers = 11;
constexpr int kCinPad = 8;          // input feature channels as stored (3 used)
constexpr int kSlab = 1024;         // voxels per weight-gradient slab

// Round-to-nearest-even FP32 -> BF16 (the rounding of the reference).
__device__ __forceinline__ __bf16 to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u = u + 0x7FFFu + ((u >> 16) & 1u);
    unsigned short h = (unsigned short)(u >> 16);
    return __builtin_bit_cast(__bf16, h);
}

struct Tensor {          // channels-last view: element (b, v, c) at b * bstride + v * stride + off + c
    float* p;
    long bstride;
    int stride;
    int off;
};

struct ConvArgs {
    const float* in;
    long in_b;
    int in_stride, in_off, cin;     // cin: multiple of 8
    float* out;
    long out_b;
    int out_stride, out_off;
    const __bf16* W;                // [cout][Kpad], k = tap * cin + ci
    int Kpad;
    const float* bias;
    const float* mask;              // MODE 1: out *= (mask > 0)
    long mask_b;
    int mask_stride, mask_off;
    int n0, n1, n2;
    long V;
    int flip;                       // 1: taps mirrored (input-gradient convolution)
};

// MODE 0: bias + ReLU; MODE 1: multiply by the mask (x > 0); MODE 2: plain.
template <int CT, int MODE>
__global__ __launch_bounds__(256) void k_conv3(ConvArgs a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4;
    const long v0 = ((long)blockIdx.x * 4 + wave) * 16;
    if (v0 >= a.V) return;                      // uniform over the wave
    const int b = blockIdx.y;
    const long v = v0 + (lane & 15);
    const bool vok = v < a.V;
    const int x = (int)(v % a.n0), y = (int)((v / a.n0) % a.n1), z = (int)(v / ((long)a.n0 * a.n1));
    const float* in = a.in + (long)b * a.in_b + a.in_off;
    v4f acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
    const int Kreal = 27 * a.cin;
    for (int k0 = 0; k0 < a.Kpad; k0 += 32) {
        const int k = k0 + 8 * grp;
        v8bf bf;
        float xs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (vok && k < Kreal) {
            const int tap = k / a.cin, ci = k - tap * a.cin;
            const int t = a.flip ? 26 - tap : tap;
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
            const int xx = x + dx, yy = y + dy, zz = z + dz;
            if (xx >= 0 && xx < a.n0 && yy >= 0 && yy < a.n1 && zz >= 0 && zz < a.n2) {
                const float* src = in + (xx + (long)a.n0 * (yy + (long)a.n1 * zz)) * a.in_stride + ci;
                const v4f p = *(const v4f*)src, q = *(const v4f*)(src + 4);
                xs[0] = p[0]; xs[1] = p[1]; xs[2] = p[2]; xs[3] = p[3];
                xs[4] = q[0]; xs[5] = q[1]; xs[6] = q[2]; xs[7] = q[3];
            }
        }
        v8bf bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const __bf16 h = to_bf16(xs[e]);
            bf[e] = h;
            bl[e] = to_bf16(xs[e] - (float)h);
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const v8bf wf = *(const v8bf*)(a.W + (long)(16 * c + (lane & 15)) * a.Kpad + k);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, bf, acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, bl, acc[c], 0, 0, 0);
        }
    }
    if (!vok) return;
    float* out = a.out + (long)b * a.out_b + v * a.out_stride + a.out_off;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int co = 16 * c + 4 * grp;
        v4f r = acc[c];
        if constexpr (MODE == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float t = r[i] + a.bias[co + i];
                r[i] = t > 0.f ? t : 0.f;
            }
        } else if constexpr (MODE == 1) {
            const v4f m = *(const v4f*)(a.mask + (long)b * a.mask_b + v * a.mask_stride + a.mask_off + co);
#pragma unroll
            for (int i = 0; i < 4; ++i) r[i] = m[i] > 0.f ? r[i] : 0.f;
        }
        *(v4f*)(out + co) = r;
    }
}

struct DwArgs {
    const float* in;
    long in_b;
    int in_stride, in_off, cin, cin_real, ntaps;   // ntaps 27 (3x3x3) or 1 (1x1x1)
    const float* g;                 // output gradient (after the activation mask)
    long g_b;
    int g_stride, cout;
    int n0, n1, n2;
    long V;
    int slabs_per_b;
    float* part;                    // [slabs][Rpad][Cpad]
    int Rpad, Cpad;
};

// Partial weight (and bias) gradients of one voxel slab: rows k = tap * cin + ci
// and one bias row k = ntaps * cin, columns = output channels.
__global__ __launch_bounds__(256) void k_conv_wgrad(DwArgs a)
{
    __shared__ v4f red[3 * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane >> 4;
    const int row = blockIdx.x * 16 + (lane & 15);
    const int col = blockIdx.y * 16 + (lane & 15);
    const int slab = blockIdx.z;
    const int b = slab / a.slabs_per_b;
    const long vs = (long)(slab - b * a.slabs_per_b) * kSlab;
    const int Kr = a.ntaps * a.cin;
    int tap = 0, ci = 0;
    bool is_w = row < Kr, is_b = row == Kr;
    if (is_w) {
        tap = row / a.cin;
        ci = row - tap * a.cin;
    }
    const int dz = a.ntaps == 27 ? tap / 9 - 1 : 0, dy = a.ntaps == 27 ? (tap / 3) % 3 - 1 : 0,
              dx = a.ntaps == 27 ? tap % 3 - 1 : 0;
    const float* in = a.in + (long)b * a.in_b + a.in_off + ci;
    const float* g = a.g + (long)b * a.g_b + col;
    const bool cok = col < a.cout;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < kSlab / 16; ++it) {
        const long v = vs + it * 16 + wave * 4 + grp;
        float av = 0.f, bv = 0.f;
        if (v < a.V) {
            if (cok) bv = g[v * a.g_stride];
            if (is_w) {
                const int x = (int)(v % a.n0), y = (int)((v / a.n0) % a.n1), z = (int)(v / ((long)a.n0 * a.n1));
                const int xx = x + dx, yy = y + dy, zz = z + dz;
                if (xx >= 0 && xx < a.n0 && yy >= 0 && yy < a.n1 && zz >= 0 && zz < a.n2)
                    av = in[(xx + (long)a.n0 * (yy + (long)a.n1 * zz)) * a.in_stride];
            } else if (is_b) {
                av = 1.f;
            }
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    if (wave > 0) red[(wave - 1) * 64 + lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    for (int w = 0; w < 3; ++w) acc += red[w * 64 + lane];
    float* dst = a.part + ((long)slab * a.Rpad + blockIdx.x * 16 + 4 * grp) * a.Cpad + col;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[(long)i * a.Cpad] = acc[i];
}

// Sum the slabs in order and scatter into the canonical gradient vector.
__global__ void k_wgrad_reduce(const float* part, int nslab, int Rpad, int Cpad, int cin, int cin_real, int ntaps,
                               int cout, float* gw, float* gb)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int Kr = ntaps * cin;
    if (i >= (long)(Kr + 1) * cout) return;
    const int row = (int)(i / cout), co = (int)(i % cout);
    float s = 0.f;
    for (int k = 0; k < nslab; ++k) s += part[((long)k * Rpad + row) * Cpad + co];
    if (row == Kr) {
        gb[co] = s;
        return;
    }
    const int tap = row / cin, ci = row - tap * cin;
    if (ci < cin_real) gw[((long)co * cin_real + ci) * ntaps + tap] = s;
}

// BF16 weights in GEMM order.  Forward: Wf[co][tap * cin_pad + ci] = W[co][ci][tap].
// Input gradient: Wb[ci][tap * cout + co] = W[co][ci][tap] (taps mirrored at use).
__global__ void k_prep_w(const float* W, int cout, int cin_real, int cin_pad, int Kpad, __bf16* Wf, __bf16* Wb,
                         int KpadB)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < (long)cout * Kpad) {
        const int co = (int)(i / Kpad), k = (int)(i % Kpad);
        float w = 0.f;
        if (k < 27 * cin_pad) {
            const int tap = k / cin_pad, ci = k % cin_pad;
            if (ci < cin_real) w = W[((long)co * cin_real + ci) * 27 + tap];
        }
        Wf[i] = to_bf16(w);
    }
    if (Wb && i < (long)cin_pad * KpadB) {
        const int ci = (int)(i / KpadB), k = (int)(i % KpadB);
        float w = 0.f;
        if (k < 27 * cout && ci < cin_real) {
            const int tap = k / cout, co = k % cout;
            w = W[((long)co * cin_real + ci) * 27 + tap];
        }
        Wb[i] = to_bf16(w);
    }
}

// Input channels: r / s, log sigma_t, sigma_s / sigma_t, zero padding.
__global__ void k_features(const double* r, const double* st, const double* ss, long N, const double* scale,
                           int media_per_rhs, float* X)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= N) return;
    const long m = media_per_rhs ? (long)b * N + i : i;
    float* d = X + ((long)b * N + i) * kCinPad;
    d[0] = (float)(r[(long)b * N + i] / scale[b]);
    d[1] = (float)log(st[m]);
    d[2] = (float)(ss[m] / st[m]);
#pragma unroll
    for (int c = 3; c < kCinPad; ++c) d[c] = 0.f;
}

// rms of each column (two passes: block partials, then one block per column).
__global__ void k_sumsq_partial(const double* x, long N, double* part, int nblk)
{
    __shared__ double sh[256];
    const int b = blockIdx.y;
    double s = 0.0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < N; i += (long)nblk * 256) {
        const double v = x[(long)b * N + i];
        s += v * v;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)b * nblk + blockIdx.x] = sh[0];
}

__global__ void k_rms_final(const double* part, int nblk, long N, double* scale)
{
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += part[(long)b * nblk + k];
    const double r = sqrt(s / (double)N);
    scale[b] = r > 0.0 ? r : 1.0;
}

__global__ void k_pool2(const float* src, long s_b, int s_stride, int s_off, int C, float* dst, long d_b, int n0,
                        int n1, int n2)
{
    const int m0 = n0 / 2, m1 = n1 / 2, m2 = n2 / 2;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= (long)m0 * m1 * m2 * C) return;
    const int c = (int)(i % C);
    const long p = i / C;
    const int x = (int)(p % m0), y = (int)((p / m0) % m1), z = (int)(p / ((long)m0 * m1));
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const long v = (2 * x + dx) + (long)n0 * ((2 * y + dy) + (long)n1 * (2 * z + dz));
                s += src[(long)b * s_b + v * s_stride + s_off + c];
            }
    dst[(long)b * d_b + p * C + c] = s * 0.125f;
}

// dst (fine grid n) channels [d_off, d_off + C) = src (coarse grid) nearest value
__global__ void k_up2(const float* src, long s_b, int C, float* dst, long d_b, int d_stride, int d_off, int n0,
                      int n1, int n2)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= (long)n0 * n1 * n2 * C) return;
    const int c = (int)(i % C);
    const long v = i / C;
    const int x = (int)(v % n0), y = (int)((v / n0) % n1), z = (int)(v / ((long)n0 * n1));
    const long p = x / 2 + (long)(n0 / 2) * (y / 2 + (long)(n1 / 2) * (z / 2));
    dst[(long)b * d_b + v * d_stride + d_off + c] = src[(long)b * s_b + p * C + c];
}

// dst (coarse) = (sum over the 8 children of g channels [g_off, g_off + C)) * (mask > 0)
__global__ void k_up2_grad_mask(const float* g, long g_b, int g_stride, int g_off, int C, const float* mask,
                                long m_b, float* dst, long d_b, int n0, int n1, int n2)
{
    const int m0 = n0 / 2, m1 = n1 / 2, m2 = n2 / 2;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= (long)m0 * m1 * m2 * C) return;
    const int c = (int)(i % C);
    const long p = i / C;
    const int x = (int)(p % m0), y = (int)((p / m0) % m1), z = (int)(p / ((long)m0 * m1));
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const long v = (2 * x + dx) + (long)n0 * ((2 * y + dy) + (long)n1 * (2 * z + dz));
                s += g[(long)b * g_b + v * g_stride + g_off + c];
            }
    dst[(long)b * d_b + p * C + c] = mask[(long)b * m_b + p * C + c] > 0.f ? s : 0.f;
}

// dst (fine, dense C) = (skip gradient + coarse gradient / 8) * (mask > 0)
__global__ void k_pool2_grad_add_mask(const float* gs, long gs_b, int gs_stride, int gs_off, const float* gp,
                                      long gp_b, const float* mask, long m_b, int m_stride, int m_off, int C,
                                      float* dst, long d_b, int n0, int n1, int n2)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= (long)n0 * n1 * n2 * C) return;
    const int c = (int)(i % C);
    const long v = i / C;
    const int x = (int)(v % n0), y = (int)((v / n0) % n1), z = (int)(v / ((long)n0 * n1));
    const long p = x / 2 + (long)(n0 / 2) * (y / 2 + (long)(n1 / 2) * (z / 2));
    const float s = gs[(long)b * gs_b + v * gs_stride + gs_off + c] + gp[(long)b * gp_b + p * C + c] * 0.125f;
    dst[(long)b * d_b + v * C + c] = mask[(long)b * m_b + v * m_stride + m_off + c] > 0.f ? s : 0.f;
}

// 1x1x1 output layer: y = sum_c w[c] x[v][c] + b
__global__ void k_head(const float* x, long x_b, int C, const float* w, const float* bias, float* y, long V)
{
    const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (v >= V) return;
    const float* xv = x + (long)b * x_b + v * C;
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += w[c] * xv[c];
    y[(long)b * V + v] = s + bias[0];
}

// Targets t = (e - r) / s (FP32) and, per column, partial sums of (y - t)^2 and t^2.
__global__ void k_loss_partial(const float* y, const double* e, const double* r, const double* scale, long V,
                               float* t, double* part, int nblk)
{
    __shared__ double s1[256], s2[256];
    const int b = blockIdx.y;
    double a = 0.0, c = 0.0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < V; i += (long)nblk * 256) {
        const float tv = (float)((e[(long)b * V + i] - r[(long)b * V + i]) / scale[b]);
        t[(long)b * V + i] = tv;
        const double d = (double)y[(long)b * V + i] - (double)tv;
        a += d * d;
        c += (double)tv * (double)tv;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((long)b * nblk + blockIdx.x) * 2] = s1[0];
        part[((long)b * nblk + blockIdx.x) * 2 + 1] = s2[0];
    }
}

// loss = mean over columns of sum (y - t)^2 / sum t^2; tt[b] = sum t^2
__global__ void k_loss_final(const double* part, int nblk, int B, double* tt, double* loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int b = 0; b < B; ++b) {
        double a = 0.0, c = 0.0;
        for (int k = 0; k < nblk; ++k) {
            a += part[((long)b * nblk + k) * 2];
            c += part[((long)b * nblk + k) * 2 + 1];
        }
        tt[b] = c > 0.0 ? c : 1.0;
        L += a / tt[b];
    }
    loss[0] = L / B;
}

// gy = 2 (y - t) / (tt B); G = w[c] gy * (x[v][c] > 0) (head and last ReLU)
__global__ void k_head_grad(const float* y, const float* t, const double* tt, int B, long V, const float* w,
                            const float* x, int C, float* gy, float* G)
{
    const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (v >= V) return;
    const float g = (float)(2.0 * ((double)y[(long)b * V + v] - (double)t[(long)b * V + v]) / (tt[b] * B));
    gy[(long)b * V + v] = g;
    const float* xv = x + ((long)b * V + v) * C;
    float* Gv = G + ((long)b * V + v) * C;
    for (int c = 0; c < C; ++c) Gv[c] = xv[c] > 0.f ? w[c] * g : 0.f;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// z = r + s y (FP64 output): the identity part of the correction plus the network's
__global__ void k_out(const float* y, const double* r, const double* scale, long V, double* z)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= V) return;
    z[(long)b * V + i] = r[(long)b * V + i] + (double)y[(long)b * V + i] * scale[b];
}

// z = r + scale * y(parent cell) on the fine grid (n0 x n1 x n2, x fastest): the
// network's output on the grid coarsened by f, extended piecewise constant.
__global__ void k_out_prolong(const float* y, const double* r, const double* scale, int n0, int n1, int n2, int f,
                              double* z)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long N = (long)n0 * n1 * n2;
    if (i >= N) return;
    const int i0 = (int)(i % n0), i1 = (int)((i / n0) % n1), i2 = (int)(i / ((long)n0 * n1));
    const int c0 = n0 / f, c1 = n1 / f;
    const long c = i0 / f + (long)c0 * (i1 / f + (long)c1 * (i2 / f));
    z[i] = r[i] + (double)y[c] * scale[0];
}

inline unsigned nblocks(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Cell averages over f x f x f blocks: y[c] = f^-3 sum of x over the fine cells of coarse
// cell c (fine grid n0 x n1 x n2, every n_a a multiple of f, x fastest; fixed summation
// order: z, then y, then x).  nrhs columns of N fine / N / f^3 coarse values.
__global__ void k_restrict(const double* __restrict__ x, int n0, int n1, int n2, int f, double* __restrict__ y)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const int c0 = n0 / f, c1 = n1 / f, c2 = n2 / f;
    const long Nc = (long)c0 * c1 * c2, N = (long)n0 * n1 * n2;
    if (i >= Nc) return;
    const int j0 = (int)(i % c0) * f, j1 = (int)((i / c0) % c1) * f, j2 = (int)(i / ((long)c0 * c1)) * f;
    const double* xb = x + (long)b * N;
    double s = 0.0;
    for (int dz = 0; dz < f; ++dz)
        for (int dy = 0; dy < f; ++dy)
            for (int dx = 0; dx < f; ++dx) s += xb[(j0 + dx) + (long)n0 * ((j1 + dy) + (long)n1 * (j2 + dz))];
    y[(long)b * Nc + i] = s / (double)(f * f * f);
}

ert_status restrict_avg(hipStream_t s, const double* x, const int n[3], int f, double* y, int nrhs)
{
    const long Nc = (long)(n[0] / f) * (n[1] / f) * (n[2] / f);
    hipLaunchKernelGGL(k_restrict, dim3(nblocks(Nc), nrhs), dim3(256), 0, s, x, n[0], n[1], n[2], f, y);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

// ----------------------------------------------------------------- host ----

struct NetLayer {
    int cin_real, cin, cout, k;     // cin: as stored (multiple of 8)
    long w_off, b_off;              // canonical parameter offsets
    int Kpad, KpadB;
    __bf16* Wf = nullptr;
    __bf16* Wb = nullptr;
};

struct NetImpl {
    ert_net_opts o;
    hipStream_t s = nullptr;
    int n[3];
    long V, V2, V4;
    int B;            // batch capacity
    int B_run = 1;    // batch of the current call
    int w1, w2, w3;
    NetLayer L[kNetLayers];
    long nparam = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *Vv = nullptr;
    long step = 0;
    // activations (per batch slot: [V][C])
    float *X = nullptr, *A1 = nullptr, *C1 = nullptr, *P1 = nullptr, *A2 = nullptr, *C2 = nullptr, *P2 = nullptr,
          *A3 = nullptr, *A3b = nullptr, *D2 = nullptr, *D2b = nullptr, *D1 = nullptr, *D1b = nullptr, *Y = nullptr;
    // gradients
    float *T = nullptr, *gY = nullptr, *Gf1 = nullptr, *Gf2 = nullptr, *GC1 = nullptr, *Gh1 = nullptr,
          *Gh2 = nullptr, *GC2 = nullptr, *Gq1 = nullptr, *Gq2 = nullptr, *part = nullptr;
    size_t part_elems = 0;
    double *scale = nullptr, *red = nullptr, *tt = nullptr, *loss = nullptr;
    int red_blk = 64;
    double* coarse = nullptr;   // restricted residual and media (3 V) for use on a finer plan grid
    std::vector<void*> allocs;

    ert_status alloc(void* pp, size_t bytes)
    {
        void** q = (void**)pp;
        if (hipMalloc(q, bytes ? bytes : 16) != hipSuccess) {
            record_error("net: device allocation failed");
            return ERT_ENOMEM;
        }
        allocs.push_back(*q);
        return ERT_OK;
    }
    ~NetImpl()
    {
        for (void* q : allocs) (void)hipFree(q);
    }
};

namespace {

ert_status conv(NetImpl* n, int li, const float* in, long in_b, int in_stride, int in_off, float* out, long out_b,
                int out_stride, int out_off, int level, int mode, bool backward, const float* mask = nullptr,
                long mask_b = 0, int mask_stride = 0, int mask_off = 0)
{
    const NetLayer& l = n->L[li];
    const int f = 1 << level;
    ConvArgs a;
    a.in = in; a.in_b = in_b; a.in_stride = in_stride; a.in_off = in_off;
    a.out = out; a.out_b = out_b; a.out_stride = out_stride; a.out_off = out_off;
    a.mask = mask; a.mask_b = mask_b; a.mask_stride = mask_stride; a.mask_off = mask_off;
    a.n0 = n->n[0] / f; a.n1 = n->n[1] / f; a.n2 = n->n[2] / f;
    a.V = (long)a.n0 * a.n1 * a.n2;
    a.bias = n->P + l.b_off;
    int cout;
    if (!backward) {
        a.cin = l.cin; a.W = l.Wf; a.Kpad = l.Kpad; a.flip = 0; cout = l.cout;
    } else {
        a.cin = l.cout; a.W = l.Wb; a.Kpad = l.KpadB; a.flip = 1; cout = l.cin;
    }
    const dim3 grid(nblocks(a.V, 64), n->B_run);
    const int ct = cout / 16;
#define ERT_CONV(CT)                                                                            \
    if (mode == 0) hipLaunchKernelGGL((k_conv3<CT, 0>), grid, dim3(256), 0, n->s, a);          \
    else if (mode == 1) hipLaunchKernelGGL((k_conv3<CT, 1>), grid, dim3(256), 0, n->s, a);     \
    else hipLaunchKernelGGL((k_conv3<CT, 2>), grid, dim3(256), 0, n->s, a);
    switch (ct) {
    case 1: ERT_CONV(1) break;
    case 2: ERT_CONV(2) break;
    case 3: ERT_CONV(3) break;
    case 4: ERT_CONV(4) break;
    case 6: ERT_CONV(6) break;
    case 8: ERT_CONV(8) break;
    default: record_error("net: unsupported channel count"); return ERT_EUNSUPPORTED;
    }
#undef ERT_CONV
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}


// Weight gradient of layer li: input activations `in` (stride/offset), output
// gradient after its mask `g` (dense cout channels), at grid level `level`.
ert_status wgrad(NetImpl* n, int li, const float* in, long in_b, int in_stride, int in_off, const float* g,
                 long g_b, int level)
{
    const NetLayer& l = n->L[li];
    const int f = 1 << level;
    DwArgs a;
    a.in = in; a.in_b = in_b; a.in_stride = in_stride; a.in_off = in_off;
    a.cin = l.cin; a.cin_real = l.cin_real; a.ntaps = l.k == 3 ? 27 : 1;
    a.g = g; a.g_b = g_b; a.g_stride = l.cout; a.cout = l.cout;
    a.n0 = n->n[0] / f; a.n1 = n->n[1] / f; a.n2 = n->n[2] / f;
    a.V = (long)a.n0 * a.n1 * a.n2;
    a.slabs_per_b = (int)((a.V + kSlab - 1) / kSlab);
    const int rows = a.ntaps * a.cin + 1;
    a.Rpad = (rows + 15) / 16 * 16;
    a.Cpad = (l.cout + 15) / 16 * 16;
    const long nslab = (long)a.slabs_per_b * n->B_run;
    if ((size_t)nslab * a.Rpad * a.Cpad > n->part_elems) {
        record_error("net: weight-gradient workspace too small");
        return ERT_EINVAL;
    }
    a.part = n->part;
    hipLaunchKernelGGL(k_conv_wgrad, dim3(a.Rpad / 16, a.Cpad / 16, (unsigned)nslab), dim3(256), 0, n->s, a);
    ERT_HIP(hipGetLastError());
    const long cnt = (long)rows * l.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(cnt)), dim3(256), 0, n->s, (const float*)n->part, (int)nslab,
                       a.Rpad, a.Cpad, a.cin, a.cin_real, a.ntaps, l.cout, n->G + l.w_off, n->G + l.b_off);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status prep_weights(NetImpl* n)
{
    for (int li = 0; li < kNetLayers; ++li) {
        NetLayer& l = n->L[li];
        if (l.k != 3) continue;
        const long cnt = std::max((long)l.cout * l.Kpad, l.Wb ? (long)l.cin * l.KpadB : 0L);
        hipLaunchKernelGGL(k_prep_w, dim3(nblocks(cnt)), dim3(256), 0, n->s, (const float*)(n->P + l.w_off), l.cout,
                           l.cin_real, l.cin, l.Kpad, l.Wf, l.Wb, l.KpadB);
        ERT_HIP(hipGetLastError());
    }
    return ERT_OK;
}

// features + column scales of r (FP64 N x B)
ert_status features(NetImpl* n, const double* r, const double* st, const double* ss, int media_per_rhs)
{
    const int B = n->B_run;
    hipLaunchKernelGGL(k_sumsq_partial, dim3(n->red_blk, B), dim3(256), 0, n->s, r, n->V, n->red, n->red_blk);
    hipLaunchKernelGGL(k_rms_final, dim3(B), dim3(64), 0, n->s, (const double*)n->red, n->red_blk, n->V, n->scale);
    hipLaunchKernelGGL(k_features, dim3(nblocks(n->V), B), dim3(256), 0, n->s, r, st, ss, n->V,
                       (const double*)n->scale, media_per_rhs, n->X);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ert_status forward(NetImpl* n)
{
    const int w1 = n->w1, w2 = n->w2, w3 = n->w3, B = n->B_run;
    const long V = n->V, V2 = n->V2, V4 = n->V4;
    const int c1s = w2 + w1, c2s = w3 + w2;
    const int n0 = n->n[0], n1 = n->n[1], n2 = n->n[2];
    ERT_TRY(conv(n, 0, n->X, V * kCinPad, kCinPad, 0, n->A1, V * w1, w1, 0, 0, 0, false));
    ERT_TRY(conv(n, 1, n->A1, V * w1, w1, 0, n->C1, V * c1s, c1s, w2, 0, 0, false));
    hipLaunchKernelGGL(k_pool2, dim3(nblocks(V2 * w1), B), dim3(256), 0, n->s, (const float*)n->C1, V * c1s, c1s, w2,
                       w1, n->P1, V2 * w1, n0, n1, n2);
    ERT_TRY(conv(n, 2, n->P1, V2 * w1, w1, 0, n->A2, V2 * w2, w2, 0, 1, 0, false));
    ERT_TRY(conv(n, 3, n->A2, V2 * w2, w2, 0, n->C2, V2 * c2s, c2s, w3, 1, 0, false));
    hipLaunchKernelGGL(k_pool2, dim3(nblocks(V4 * w2), B), dim3(256), 0, n->s, (const float*)n->C2, V2 * c2s, c2s, w3,
                       w2, n->P2, V4 * w2, n0 / 2, n1 / 2, n2 / 2);
    ERT_TRY(conv(n, 4, n->P2, V4 * w2, w2, 0, n->A3, V4 * w3, w3, 0, 2, 0, false));
    ERT_TRY(conv(n, 5, n->A3, V4 * w3, w3, 0, n->A3b, V4 * w3, w3, 0, 2, 0, false));
    hipLaunchKernelGGL(k_up2, dim3(nblocks(V2 * w3), B), dim3(256), 0, n->s, (const float*)n->A3b, V4 * w3, w3, n->C2,
                       V2 * c2s, c2s, 0, n0 / 2, n1 / 2, n2 / 2);
    ERT_TRY(conv(n, 6, n->C2, V2 * c2s, c2s, 0, n->D2, V2 * w2, w2, 0, 1, 0, false));
    ERT_TRY(conv(n, 7, n->D2, V2 * w2, w2, 0, n->D2b, V2 * w2, w2, 0, 1, 0, false));
    hipLaunchKernelGGL(k_up2, dim3(nblocks(V * w2), B), dim3(256), 0, n->s, (const float*)n->D2b, V2 * w2, w2, n->C1,
                       V * c1s, c1s, 0, n0, n1, n2);
    ERT_TRY(conv(n, 8, n->C1, V * c1s, c1s, 0, n->D1, V * w1, w1, 0, 0, 0, false));
    ERT_TRY(conv(n, 9, n->D1, V * w1, w1, 0, n->D1b, V * w1, w1, 0, 0, 0, false));
    hipLaunchKernelGGL(k_head, dim3(nblocks(V), B), dim3(256), 0, n->s, (const float*)n->D1b, V * w1, w1,
                       (const float*)(n->P + n->L[10].w_off), (const float*)(n->P + n->L[10].b_off), n->Y, V);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

// loss and gradient (n->G) for corrections e of residuals r (FP64 N x B), after forward()
ert_status backward(NetImpl* n, const double* r, const double* e)
{
    const int w1 = n->w1, w2 = n->w2, w3 = n->w3, B = n->B_run;
    const long V = n->V, V2 = n->V2, V4 = n->V4;
    const int c1s = w2 + w1, c2s = w3 + w2;
    const int n0 = n->n[0], n1 = n->n[1], n2 = n->n[2];
    hipLaunchKernelGGL(k_loss_partial, dim3(n->red_blk, B), dim3(256), 0, n->s, (const float*)n->Y, e, r,
                       (const double*)n->scale, V, n->T, n->red, n->red_blk);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, n->s, (const double*)n->red, n->red_blk, B, n->tt, n->loss);
    // head: gY and the masked gradient of L10's output (Gf1)
    hipLaunchKernelGGL(k_head_grad, dim3(nblocks(V), B), dim3(256), 0, n->s, (const float*)n->Y, (const float*)n->T,
                       (const double*)n->tt, B, V, (const float*)(n->P + n->L[10].w_off), (const float*)n->D1b, w1,
                       n->gY, n->Gf1);
    ERT_HIP(hipGetLastError());
    ERT_TRY(wgrad(n, 10, n->D1b, V * w1, w1, 0, n->gY, V, 0));
    // L10
    ERT_TRY(wgrad(n, 9, n->D1, V * w1, w1, 0, n->Gf1, V * w1, 0));
    ERT_TRY(conv(n, 9, n->Gf1, V * w1, w1, 0, n->Gf2, V * w1, w1, 0, 0, 1, true, n->D1, V * w1, w1, 0));
    // L9 (input: concat [up(D2b), s1])
    ERT_TRY(wgrad(n, 8, n->C1, V * c1s, c1s, 0, n->Gf2, V * w1, 0));
    ERT_TRY(conv(n, 8, n->Gf2, V * w1, w1, 0, n->GC1, V * c1s, c1s, 0, 0, 2, true));
    hipLaunchKernelGGL(k_up2_grad_mask, dim3(nblocks(V2 * w2), B), dim3(256), 0, n->s, (const float*)n->GC1, V * c1s,
                       c1s, 0, w2, (const float*)n->D2b, V2 * w2, n->Gh1, V2 * w2, n0, n1, n2);
    // L8
    ERT_TRY(wgrad(n, 7, n->D2, V2 * w2, w2, 0, n->Gh1, V2 * w2, 1));
    ERT_TRY(conv(n, 7, n->Gh1, V2 * w2, w2, 0, n->Gh2, V2 * w2, w2, 0, 1, 1, true, n->D2, V2 * w2, w2, 0));
    // L7 (input: concat [up(A3b), s2])
    ERT_TRY(wgrad(n, 6, n->C2, V2 * c2s, c2s, 0, n->Gh2, V2 * w2, 1));
    ERT_TRY(conv(n, 6, n->Gh2, V2 * w2, w2, 0, n->GC2, V2 * c2s, c2s, 0, 1, 2, true));
    hipLaunchKernelGGL(k_up2_grad_mask, dim3(nblocks(V4 * w3), B), dim3(256), 0, n->s, (const float*)n->GC2,
                       V2 * c2s, c2s, 0, w3, (const float*)n->A3b, V4 * w3, n->Gq1, V4 * w3, n0 / 2, n1 / 2, n2 / 2);
    // L6
    ERT_TRY(wgrad(n, 5, n->A3, V4 * w3, w3, 0, n->Gq1, V4 * w3, 2));
    ERT_TRY(conv(n, 5, n->Gq1, V4 * w3, w3, 0, n->Gq2, V4 * w3, w3, 0, 2, 1, true, n->A3, V4 * w3, w3, 0));
    // L5 (input: pool(s2)); its input gradient goes to Gq1 (w2 channels)
    ERT_TRY(wgrad(n, 4, n->P2, V4 * w2, w2, 0, n->Gq2, V4 * w3, 2));
    ERT_TRY(conv(n, 4, n->Gq2, V4 * w3, w3, 0, n->Gq1, V4 * w2, w2, 0, 2, 2, true));
    hipLaunchKernelGGL(k_pool2_grad_add_mask, dim3(nblocks(V2 * w2), B), dim3(256), 0, n->s, (const float*)n->GC2,
                       V2 * c2s, c2s, w3, (const float*)n->Gq1, V4 * w2, (const float*)n->C2, V2 * c2s, c2s, w3, w2,
                       n->Gh1, V2 * w2, n0 / 2, n1 / 2, n2 / 2);
    // L4
    ERT_TRY(wgrad(n, 3, n->A2, V2 * w2, w2, 0, n->Gh1, V2 * w2, 1));
    ERT_TRY(conv(n, 3, n->Gh1, V2 * w2, w2, 0, n->Gh2, V2 * w2, w2, 0, 1, 1, true, n->A2, V2 * w2, w2, 0));
    // L3 (input: pool(s1)); input gradient to Gh1 (w1 channels)
    ERT_TRY(wgrad(n, 2, n->P1, V2 * w1, w1, 0, n->Gh2, V2 * w2, 1));
    ERT_TRY(conv(n, 2, n->Gh2, V2 * w2, w2, 0, n->Gh1, V2 * w1, w1, 0, 1, 2, true));
    hipLaunchKernelGGL(k_pool2_grad_add_mask, dim3(nblocks(V * w1), B), dim3(256), 0, n->s, (const float*)n->GC1,
                       V * c1s, c1s, w2, (const float*)n->Gh1, V2 * w1, (const float*)n->C1, V * c1s, c1s, w2, w1,
                       n->Gf1, V * w1, n0, n1, n2);
    // L2
    ERT_TRY(wgrad(n, 1, n->A1, V * w1, w1, 0, n->Gf1, V * w1, 0));
    ERT_TRY(conv(n, 1, n->Gf1, V * w1, w1, 0, n->Gf2, V * w1, w1, 0, 0, 1, true, n->A1, V * w1, w1, 0));
    // L1 (features; no input gradient)
    ERT_TRY(wgrad(n, 0, n->X, V * kCinPad, kCinPad, 0, n->Gf2, V * w1, 0));
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

}  // namespace

// Solver-side use: z = M(r) for one residual column on the plan's media (grid pn).
// A network on the plan's grid coarsened by f (pn = f n) acts on the cell averages of
// r, sigma_t and sigma_s over f^3 blocks, and its output is extended piecewise
// constant: z = r + P(s_c y(R r)).
ert_status net_precond(NetImpl* n, const double* r, const double* st, const double* ss, double* z, hipStream_t s,
                       const int* pn)
{
    const int f = pn[0] / n->n[0];
    hipStream_t keep = n->s;
    n->s = s;
    n->B_run = 1;
    ert_status st_ = ERT_OK;
    if (f > 1) {
        if (!n->coarse) st_ = n->alloc(&n->coarse, 3 * (size_t)n->V * sizeof(double));
        if (st_ == ERT_OK) st_ = restrict_avg(s, r, pn, f, n->coarse, 1);
        if (st_ == ERT_OK) st_ = restrict_avg(s, st, pn, f, n->coarse + n->V, 1);
        if (st_ == ERT_OK) st_ = restrict_avg(s, ss, pn, f, n->coarse + 2 * n->V, 1);
        if (st_ == ERT_OK) st_ = features(n, n->coarse, n->coarse + n->V, n->coarse + 2 * n->V, 0);
    } else {
        st_ = features(n, r, st, ss, 0);
    }
    if (st_ == ERT_OK) st_ = forward(n);
    if (st_ == ERT_OK) {
        if (f > 1) {
            const long N = (long)pn[0] * pn[1] * pn[2];
            hipLaunchKernelGGL(k_out_prolong, dim3(nblocks(N), 1), dim3(256), 0, s, (const float*)n->Y, r,
                               (const double*)n->scale, pn[0], pn[1], pn[2], f, z);
        } else {
            hipLaunchKernelGGL(k_out, dim3(nblocks(n->V), 1), dim3(256), 0, s, (const float*)n->Y, r,
                               (const double*)n->scale, n->V, z);
        }
        if (hipGetLastError() != hipSuccess) st_ = ERT_EDEVICE;
    }
    n->s = keep;
    return st_;
}

const int* net_grid(const NetImpl* n) { return n->n; }

}  // namespace ertvie

using namespace ertvie;

struct ert_net_s : public NetImpl {};

namespace ertvie {
NetImpl* net_impl(ert_net_t net) { return static_cast<NetImpl*>(net); }
}  // namespace ertvie

extern "C" {

ERT_API long ert_net_param_count(const ert_net_opts* o)
{
    if (!o) return -1;
    const int w1 = o->width[0] ? o->width[0] : 16, w2 = o->width[1] ? o->width[1] : 32,
              w3 = o->width[2] ? o->width[2] : 64;
    const int sh[kNetLayers][3] = {{w1, 3, 3}, {w1, w1, 3}, {w2, w1, 3}, {w2, w2, 3}, {w3, w2, 3}, {w3, w3, 3},
                                   {w2, w3 + w2, 3}, {w2, w2, 3}, {w1, w2 + w1, 3}, {w1, w1, 3}, {1, w1, 1}};
    long c = 0;
    for (int i = 0; i < kNetLayers; ++i) c += (long)sh[i][0] * sh[i][1] * sh[i][2] * sh[i][2] * sh[i][2] + sh[i][0];
    return c;
}

ERT_API ert_status ert_net_create(const ert_net_opts* o, void* hip_stream, ert_net_t* out)
{
    if (!o || !out) {
        record_error("ert_net_create: null argument");
        return ERT_EINVAL;
    }
    *out = nullptr;
    const int w1 = o->width[0] ? o->width[0] : 16, w2 = o->width[1] ? o->width[1] : 32,
              w3 = o->width[2] ? o->width[2] : 64;
    if (o->dim != 3) {
        record_error("ert_net_create: the network is three-dimensional (dim must be 3)");
        return o->dim == 2 ? ERT_EUNSUPPORTED : ERT_EINVAL;
    }
    for (int a = 0; a < 3; ++a)
        if (o->n[a] < 4 || o->n[a] % 4 != 0) {
            record_error("ert_net_create: every grid extent must be a positive multiple of 4");
            return ERT_EINVAL;
        }
    if (w1 % 16 || w2 % 16 || w3 % 16 || w1 > 128 || w2 > 128 || w3 > 128 || w1 < 16 || w2 < 16 || w3 < 16) {
        record_error("ert_net_create: widths must be multiples of 16 in [16, 128]");
        return ERT_EINVAL;
    }
    for (int i = 0; i < 4; ++i)
        if (o->reserved[i]) {
            record_error("ert_net_create: reserved fields must be 0");
            return ERT_EINVAL;
        }
    const int B = o->batch_max > 0 ? o->batch_max : 1;
    ert_net_s* n = new (std::nothrow) ert_net_s();
    if (!n) return ERT_ENOMEM;
    n->o = *o;
    n->s = (hipStream_t)hip_stream;
    for (int a = 0; a < 3; ++a) n->n[a] = o->n[a];
    n->V = (long)o->n[0] * o->n[1] * o->n[2];
    n->V2 = n->V / 8;
    n->V4 = n->V / 64;
    n->B = B;
    n->w1 = w1; n->w2 = w2; n->w3 = w3;
    const int sh[kNetLayers][3] = {{w1, 3, 3}, {w1, w1, 3}, {w2, w1, 3}, {w2, w2, 3}, {w3, w2, 3}, {w3, w3, 3},
                                   {w2, w3 + w2, 3}, {w2, w2, 3}, {w1, w2 + w1, 3}, {w1, w1, 3}, {1, w1, 1}};
    long off = 0;
    ert_status st = ERT_OK;
    for (int i = 0; i < kNetLayers && st == ERT_OK; ++i) {
        NetLayer& l = n->L[i];
        l.cout = sh[i][0];
        l.cin_real = sh[i][1];
        l.cin = i == 0 ? kCinPad : l.cin_real;
        l.k = sh[i][2];
        l.w_off = off;
        off += (long)l.cout * l.cin_real * l.k * l.k * l.k;
        l.b_off = off;
        off += l.cout;
        if (l.k == 3) {
            l.Kpad = (27 * l.cin + 31) / 32 * 32;
            st = n->alloc(&l.Wf, (size_t)l.cout * l.Kpad * sizeof(__bf16));
            if (i > 0 && st == ERT_OK) {
                l.KpadB = (27 * l.cout + 31) / 32 * 32;
                st = n->alloc(&l.Wb, (size_t)l.cin * l.KpadB * sizeof(__bf16));
            }
        }
    }
    n->nparam = off;
    const long V = n->V, V2 = n->V2, V4 = n->V4;
    auto fl = [&](float** p, long elems) {
        if (st == ERT_OK) st = n->alloc(p, (size_t)elems * B * sizeof(float));
    };
    if (st == ERT_OK) st = n->alloc(&n->P, n->nparam * sizeof(float));
    if (st == ERT_OK) st = n->alloc(&n->G, n->nparam * sizeof(float));
    if (st == ERT_OK) st = n->alloc(&n->M, n->nparam * sizeof(float));
    if (st == ERT_OK) st = n->alloc(&n->Vv, n->nparam * sizeof(float));
    fl(&n->X, V * kCinPad);
    fl(&n->A1, V * w1);
    fl(&n->C1, V * (w2 + w1));
    fl(&n->P1, V2 * w1);
    fl(&n->A2, V2 * w2);
    fl(&n->C2, V2 * (w3 + w2));
    fl(&n->P2, V4 * w2);
    fl(&n->A3, V4 * w3);
    fl(&n->A3b, V4 * w3);
    fl(&n->D2, V2 * w2);
    fl(&n->D2b, V2 * w2);
    fl(&n->D1, V * w1);
    fl(&n->D1b, V * w1);
    fl(&n->Y, V);
    fl(&n->T, V);
    fl(&n->gY, V);
    fl(&n->Gf1, V * w1);
    fl(&n->Gf2, V * w1);
    fl(&n->GC1, V * (w2 + w1));
    fl(&n->Gh1, V2 * std::max(w1, w2));
    fl(&n->Gh2, V2 * w2);
    fl(&n->GC2, V2 * (w3 + w2));
    fl(&n->Gq1, V4 * std::max(w2, w3));
    fl(&n->Gq2, V4 * w3);
    // weight-gradient slabs: the largest layer
    size_t need = 0;
    for (int i = 0; i < kNetLayers; ++i) {
        const NetLayer& l = n->L[i];
        const int level = (i < 2 || i >= 8) ? 0 : ((i < 4 || i >= 6) ? 1 : 2);
        const long Vl = V >> (3 * level);
        const long slabs = (Vl + kSlab - 1) / kSlab * B;
        const long rows = (long)(l.k == 3 ? 27 : 1) * l.cin + 1;
        need = std::max(need, (size_t)slabs * ((rows + 15) / 16 * 16) * ((l.cout + 15) / 16 * 16));
    }
    if (st == ERT_OK) st = n->alloc(&n->part, need * sizeof(float));
    n->part_elems = need;
    if (st == ERT_OK) st = n->alloc(&n->scale, (size_t)B * sizeof(double));
    if (st == ERT_OK) st = n->alloc(&n->tt, (size_t)B * sizeof(double));
    if (st == ERT_OK) st = n->alloc(&n->loss, sizeof(double));
    if (st == ERT_OK) st = n->alloc(&n->red, (size_t)B * n->red_blk * 2 * sizeof(double));
    if (st == ERT_OK && (hipMemsetAsync(n->P, 0, n->nparam * sizeof(float), n->s) != hipSuccess ||
                         hipMemsetAsync(n->M, 0, n->nparam * sizeof(float), n->s) != hipSuccess ||
                         hipMemsetAsync(n->Vv, 0, n->nparam * sizeof(float), n->s) != hipSuccess))
        st = ERT_EDEVICE;
    if (st != ERT_OK) {
        delete n;
        return st;
    }
    *out = n;
    return ERT_OK;
}

ERT_API long ert_net_size(ert_net_t net) { return net ? net->nparam : -1; }

ERT_API ert_status ert_net_set_params(ert_net_t net, const float* params)
{
    if (!net || !params) {
        record_error("ert_net_set_params: null argument");
        return ERT_EINVAL;
    }
    ERT_HIP(hipMemcpyAsync(net->P, params, net->nparam * sizeof(float), hipMemcpyHostToDevice, net->s));
    ERT_HIP(hipMemsetAsync(net->M, 0, net->nparam * sizeof(float), net->s));
    ERT_HIP(hipMemsetAsync(net->Vv, 0, net->nparam * sizeof(float), net->s));
    net->step = 0;
    ERT_TRY(prep_weights(net));
    ERT_HIP(hipStreamSynchronize(net->s));
    return ERT_OK;
}

ERT_API ert_status ert_net_get_params(ert_net_t net, float* params)
{
    if (!net || !params) {
        record_error("ert_net_get_params: null argument");
        return ERT_EINVAL;
    }
    ERT_HIP(hipMemcpyAsync(params, net->P, net->nparam * sizeof(float), hipMemcpyDeviceToHost, net->s));
    ERT_HIP(hipStreamSynchronize(net->s));
    return ERT_OK;
}

static ert_status net_check(ert_net_t net, const void* a, const void* b, int batch, const char* who)
{
    if (!net || !a || !b) {
        record_error(who);
        return ERT_EINVAL;
    }
    if (batch < 1 || batch > net->B) {
        record_error("net: batch outside 1..batch_max");
        return ERT_EINVAL;
    }
    return ERT_OK;
}

ERT_API ert_status ert_net_forward(ert_net_t net, const double* r, const double* sigma_t, const double* sigma_s,
                                   double* z, int batch)
{
    ERT_TRY(net_check(net, r, z, batch, "ert_net_forward: null argument"));
    if (!sigma_t || !sigma_s) {
        record_error("ert_net_forward: null medium");
        return ERT_EINVAL;
    }
    net->B_run = batch;
    ERT_TRY(features(net, r, sigma_t, sigma_s, 1));
    ERT_TRY(forward(net));
    hipLaunchKernelGGL(k_out, dim3(nblocks(net->V), batch), dim3(256), 0, net->s, (const float*)net->Y, r,
                       (const double*)net->scale, net->V, z);
    ERT_HIP(hipGetLastError());
    return ERT_OK;
}

ERT_API ert_status ert_net_grad(ert_net_t net, const double* r, const double* e, const double* sigma_t,
                                const double* sigma_s, int batch, double* loss, float* grad)
{
    ERT_TRY(net_check(net, r, e, batch, "ert_net_grad: null argument"));
    if (!sigma_t || !sigma_s) {
        record_error("ert_net_grad: null medium");
        return ERT_EINVAL;
    }
    net->B_run = batch;
    ERT_TRY(features(net, r, sigma_t, sigma_s, 1));
    ERT_TRY(forward(net));
    ERT_TRY(backward(net, r, e));
    if (loss) ERT_HIP(hipMemcpyAsync(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->s));
    if (grad) ERT_HIP(hipMemcpyAsync(grad, net->G, net->nparam * sizeof(float), hipMemcpyDeviceToHost, net->s));
    ERT_HIP(hipStreamSynchronize(net->s));
    return ERT_OK;
}

ERT_API ert_status ert_net_train_step(ert_net_t net, const double* r, const double* e, const double* sigma_t,
                                      const double* sigma_s, int batch, const ert_net_train_opts* opts, double* loss)
{
    ERT_TRY(net_check(net, r, e, batch, "ert_net_train_step: null argument"));
    if (!sigma_t || !sigma_s || !opts) {
        record_error("ert_net_train_step: null medium or options");
        return ERT_EINVAL;
    }
    const double lr = opts->lr > 0 ? opts->lr : 1e-3, b1 = opts->beta1 > 0 ? opts->beta1 : 0.9,
                 b2 = opts->beta2 > 0 ? opts->beta2 : 0.999, eps = opts->eps > 0 ? opts->eps : 1e-8;
    if (!(lr < 1.0) || !(b1 < 1.0) || !(b2 < 1.0)) {
        record_error("ert_net_train_step: lr, beta1 and beta2 must lie in (0, 1)");
        return ERT_EINVAL;
    }
    net->B_run = batch;
    ERT_TRY(features(net, r, sigma_t, sigma_s, 1));
    ERT_TRY(forward(net));
    ERT_TRY(backward(net, r, e));
    net->step += 1;
    const float c1 = (float)(1.0 - std::pow(b1, (double)net->step)), c2 = (float)(1.0 - std::pow(b2, (double)net->step));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(net->nparam)), dim3(256), 0, net->s, net->P, (const float*)net->G, net->M,
                       net->Vv, net->nparam, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    ERT_HIP(hipGetLastError());
    ERT_TRY(prep_weights(net));
    if (loss) {
        ERT_HIP(hipMemcpyAsync(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->s));
        ERT_HIP(hipStreamSynchronize(net->s));
    }
    return ERT_OK;
}

ERT_API void ert_net_destroy(ert_net_t net) { delete net; }

}  // extern "C"
