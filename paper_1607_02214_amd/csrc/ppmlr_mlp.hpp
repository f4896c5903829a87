// Small MLP that proposes the starting pressure of the interface Riemann
// solver's Newton iteration (the learned guess of the paper's batched /
// learned variants): 14 inputs (left and right primitive states, normalised
// by the pair means), two hidden layers of 64 with the tanh form of GELU
// (Hendrycks & Gimpel 2016), 2 outputs (star pressure and velocity as
// residuals on the plain linear guess).
//
// BF16 operands, FP32 accumulation, on the gfx950 matrix cores
// (v_mfma_f32_16x16x16_bf16).  Every product is computed transposed, with
// samples along the N (column) dimension:  Z^T = W^T H^T.  Then the FP32
// accumulator tile of one layer (lane l: column l%16, rows 4*(l/16)+i) has
// exactly the register layout of the B operand of the next layer (lane l:
// column l%16, k = 4*(l/16)+i), so activations never leave registers in the
// forward pass.  Weights are pre-packed into A-operand fragments (64 lanes x
// 4 BF16 per 16x16 tile, one coalesced 8-byte load per lane).
//
// Parameter vector theta (FP32, 5250 values): W1[14][64], b1[64],
// W2[64][64], b2[64], W3[64][2], b3[2], row-major (input index first).
#pragma once
#include <hip/hip_runtime.h>

namespace ppmlr {
namespace mlp {

constexpr int kIn = 14, kH = 64, kOut = 2;
constexpr int kOffW1 = 0, kOffB1 = kIn * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kOut, kNPar = kOffB3 + kOut;
static_assert(kNPar == 5250, "parameter count");

// packed fragment tiles (each 16x16 tile = 256 BF16)
constexpr int kTA1 = 0;            // W1^T: 4 (m) x 1 (k)   forward layer 1
constexpr int kTA2 = 4;            // W2^T: 4 x 4           forward layer 2
constexpr int kTA3 = 20;           // W3^T: 1 x 4           forward layer 3
constexpr int kTB3 = 24;           // W3  : 4 x 1           backward through layer 3
constexpr int kTB2 = 28;           // W2  : 4 x 4           backward through layer 2
constexpr int kTiles = 44;
constexpr int kFwdTiles = 24;      // the forward pass needs tiles [0, 24)
constexpr int kRecord = 28;        // floats per harvested interface record

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (quiet NaN kept NaN)
__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    bf16x4 r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// tanh-form GELU, written through the logistic function:
// x/2 (1 + tanh(u)) = x * sigma(2u),  u = sqrt(2/pi) (x + 0.044715 x^3)
constexpr float kGc = 0.7978845608028654f, kGa = 0.044715f;
__device__ __forceinline__ float gelu(float x)
{
    const float u = kGc * (x + kGa * x * x * x);
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * u));
    return x * s;
}
// derivative: sigma(2u) + x * 2 sigma (1 - sigma) * du/dx
__device__ __forceinline__ float gelu_grad(float x)
{
    const float u = kGc * (x + kGa * x * x * x);
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * u));
    return s + x * 2.0f * s * (1.0f - s) * kGc * (1.0f + 3.0f * kGa * x * x);
}

// Value of fragment element (tile t, lane l, item i) of the packed set.
__device__ inline float frag_value(const float *th, int t, int l, int i)
{
    const int r = l & 15, kk = 4 * (l >> 4) + i;
    if (t < kTA2) {                        // W1^T: m = hidden, k = input feature
        const int m = t * 16 + r, k = kk;
        return k < kIn ? th[kOffW1 + k * kH + m] : 0.0f;
    }
    if (t < kTA3) {                        // W2^T: m = out hidden, k = in hidden
        const int u = t - kTA2, m = (u >> 2) * 16 + r, k = (u & 3) * 16 + kk;
        return th[kOffW2 + k * kH + m];
    }
    if (t < kTB3) {                        // W3^T: m = output, k = hidden
        const int m = r, k = (t - kTA3) * 16 + kk;
        return m < kOut ? th[kOffW3 + k * kOut + m] : 0.0f;
    }
    if (t < kTB2) {                        // W3: m = hidden, k = output
        const int m = (t - kTB3) * 16 + r, k = kk;
        return k < kOut ? th[kOffW3 + m * kOut + k] : 0.0f;
    }
    {                                      // W2: m = in hidden, k = out hidden
        const int u = t - kTB2, m = (u >> 2) * 16 + r, k = (u & 3) * 16 + kk;
        return th[kOffW2 + m * kH + k];
    }
}

// Pack theta into BF16 fragments: frag[(t * 64 + l) * 4 + i].
__global__ void pack_kernel(const float *__restrict__ theta, unsigned short *__restrict__ frag, int tiles)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tiles * 256) return;
    const int t = idx >> 8, l = (idx >> 2) & 63, i = idx & 3;
    frag[idx] = f2bf(frag_value(theta, t, l, i));
}

__device__ __forceinline__ bf16x4 load_frag(const unsigned short *frag, int t, int lane)
{
    return *reinterpret_cast<const bf16x4 *>(frag + ((size_t)t * 64 + lane) * 4);
}

// Forward pass of one wave over 64 samples.  F: BF16 features, row-major
// [64][16] (columns 14, 15 zero), in LDS.  Writes the two outputs of sample s
// to out[s * ldo + o] (lanes 0..15 hold them).  Must be called by all 64
// lanes of the wave.  The 64 samples are taken as four tiles of 16, one after
// the other, so that only one tile's activations are live (this runs inside
// the sweep, next to the solver's own registers); the weight fragments are
// re-read per tile from the L2-resident packed buffer.
__device__ __forceinline__ void forward_wave(const unsigned short *F, const unsigned short *frag,
                                             const float *__restrict__ theta, float *out, int ldo)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int st = 0; st < 4; ++st) {
        // keeps the weight loads inside the loop (not hoisted into registers)
        asm volatile("" ::: "memory");
        const bf16x4 xb = *reinterpret_cast<const bf16x4 *>(F + (st * 16 + r) * 16 + 4 * q);
        // layer 1: Z1^T[64 x 16] = W1^T[64 x 16] X^T[16 x 16]
        bf16x4 h1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4 z = mfma(load_frag(frag, kTA1 + mt, lane), xb, zero);
            const float *b1 = theta + kOffB1 + mt * 16 + 4 * q;
            h1[mt] = pack4(gelu(z[0] + b1[0]), gelu(z[1] + b1[1]), gelu(z[2] + b1[2]), gelu(z[3] + b1[3]));
        }
        // layer 2: Z2^T = W2^T H1^T (weight loads kept per output tile, so
        // that at most four fragments are in flight)
        bf16x4 h2[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            asm volatile("" ::: "memory");
            f32x4 acc = zero;
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) acc = mfma(load_frag(frag, kTA2 + mt * 4 + kt, lane), h1[kt], acc);
            const float *b2 = theta + kOffB2 + mt * 16 + 4 * q;
            h2[mt] = pack4(gelu(acc[0] + b2[0]), gelu(acc[1] + b2[1]), gelu(acc[2] + b2[2]), gelu(acc[3] + b2[3]));
        }
        // layer 3: O^T[16 x 16] = W3^T[16 x 64] H2^T (rows 0, 1 valid)
        f32x4 o = zero;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) o = mfma(load_frag(frag, kTA3 + kt, lane), h2[kt], o);
        if (q == 0) {
            out[(st * 16 + r) * ldo + 0] = o[0] + theta[kOffB3];
            out[(st * 16 + r) * ldo + 1] = o[1] + theta[kOffB3 + 1];
        }
    }
}

// Forward over n samples: one wave per 64 samples.
__global__ void __launch_bounds__(64) forward_kernel(const float *__restrict__ X, int ldx, int n,
                                                     const unsigned short *__restrict__ frag,
                                                     const float *__restrict__ theta, float *__restrict__ Y, int ldy)
{
    __shared__ __align__(16) unsigned short F[64 * 16];
    __shared__ float O[64 * 2];
    const int lane = threadIdx.x;
    const long long s = (long long)blockIdx.x * 64 + lane;
#pragma unroll
    for (int k = 0; k < 16; ++k) F[lane * 16 + k] = (s < n && k < kIn) ? f2bf(X[s * ldx + k]) : (unsigned short)0;
    __syncthreads();
    forward_wave(F, frag, theta, O, 2);
    __syncthreads();
    if (s < n) {
        Y[s * ldy + 0] = O[lane * 2 + 0];
        Y[s * ldy + 1] = O[lane * 2 + 1];
    }
}

// Loss and gradient of L = (1 / 2n) sum (o - y)^2 over one wave's 64 samples
// (rows beyond n contribute nothing).  Writes the partial gradient of this
// workgroup, in theta order, and its partial loss to part[kNPar].  The
// backward pass uses the same BF16 operands / FP32 accumulation; the GELU
// derivatives are kept in BF16.
__global__ void __launch_bounds__(64) grad_kernel(const float *__restrict__ X, int ldx, const float *__restrict__ Yt,
                                                  int ldy, int n, const unsigned short *__restrict__ frag,
                                                  const float *__restrict__ theta, float *__restrict__ partials)
{
    __shared__ __align__(16) unsigned short XT[16 * 64];   // [f][s]
    __shared__ __align__(16) unsigned short H1T[64 * 64];  // [hid][s]
    __shared__ __align__(16) unsigned short H2T[64 * 64];
    __shared__ __align__(16) unsigned short D2T[64 * 64];  // dZ2^T
    __shared__ __align__(16) unsigned short D1T[64 * 64];  // dZ1^T
    __shared__ __align__(16) unsigned short DOT[16 * 64];  // dO^T, rows >= 2 zero
    __shared__ __align__(16) bf16x4 G1F[16 * 64];          // gelu'(Z1), fragment order
    __shared__ __align__(16) bf16x4 G2F[16 * 64];
    __shared__ float red[64];
    const int lane = threadIdx.x;
    const int r = lane & 15, q = lane >> 4;
    const long long s0 = (long long)blockIdx.x * 64;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    float *part = partials + (size_t)blockIdx.x * (kNPar + 1);
    for (int k = 0; k < 16; ++k) {
        const long long s = s0 + lane;
        XT[k * 64 + lane] = (s < n && k < kIn) ? f2bf(X[s * ldx + k]) : (unsigned short)0;
    }
    __syncthreads();
    auto fragT = [&](const unsigned short *M, int row0, int kt) -> bf16x4 {   // M[row][s]: rows row0 + r
        return *reinterpret_cast<const bf16x4 *>(M + (row0 + r) * 64 + kt * 16 + 4 * q);
    };
    // ---- forward (transposed), keeping activations and GELU derivatives
    bf16x4 xb[4];
    for (int st = 0; st < 4; ++st)
        for (int i = 0; i < 4; ++i) xb[st][i] = (short)XT[(4 * q + i) * 64 + st * 16 + r];
    bf16x4 h1[4][4];
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x4 a = load_frag(frag, kTA1 + mt, lane);
        for (int st = 0; st < 4; ++st) {
            f32x4 z = mfma(a, xb[st], zero);
            for (int i = 0; i < 4; ++i) z[i] += theta[kOffB1 + mt * 16 + 4 * q + i];
            G1F[(mt * 4 + st) * 64 + lane] = pack4(gelu_grad(z[0]), gelu_grad(z[1]), gelu_grad(z[2]), gelu_grad(z[3]));
            h1[mt][st] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
            for (int i = 0; i < 4; ++i) H1T[(mt * 16 + 4 * q + i) * 64 + st * 16 + r] = (unsigned short)h1[mt][st][i];
        }
    }
    bf16x4 h2[4][4];
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc[4] = {zero, zero, zero, zero};
        for (int kt = 0; kt < 4; ++kt) {
            const bf16x4 a = load_frag(frag, kTA2 + mt * 4 + kt, lane);
            for (int st = 0; st < 4; ++st) acc[st] = mfma(a, h1[kt][st], acc[st]);
        }
        for (int st = 0; st < 4; ++st) {
            f32x4 z = acc[st];
            for (int i = 0; i < 4; ++i) z[i] += theta[kOffB2 + mt * 16 + 4 * q + i];
            G2F[(mt * 4 + st) * 64 + lane] = pack4(gelu_grad(z[0]), gelu_grad(z[1]), gelu_grad(z[2]), gelu_grad(z[3]));
            h2[mt][st] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
            for (int i = 0; i < 4; ++i) H2T[(mt * 16 + 4 * q + i) * 64 + st * 16 + r] = (unsigned short)h2[mt][st][i];
        }
    }
    f32x4 o[4] = {zero, zero, zero, zero};
    for (int kt = 0; kt < 4; ++kt) {
        const bf16x4 a = load_frag(frag, kTA3 + kt, lane);
        for (int st = 0; st < 4; ++st) o[st] = mfma(a, h2[kt][st], o[st]);
    }
    // ---- output error dO = (o - y) / n (rows 0, 1 of the output tile), loss
    const float inv_n = 1.0f / (float)n;
    float sq = 0.0f;
    bf16x4 dob[4];
    float db3[2] = {0.0f, 0.0f};
    for (int st = 0; st < 4; ++st) {
        const long long ss = s0 + st * 16 + r;
        float d[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (q == 0 && ss < n) {
            for (int k = 0; k < kOut; ++k) {
                const float e = o[st][k] + theta[kOffB3 + k] - Yt[ss * ldy + k];
                sq += e * e;
                d[k] = e * inv_n;
            }
        }
        db3[0] += d[0];
        db3[1] += d[1];
        dob[st] = pack4(d[0], d[1], d[2], d[3]);
        for (int i = 0; i < 4; ++i) DOT[(4 * q + i) * 64 + st * 16 + r] = (unsigned short)dob[st][i];
    }
    // ---- through layer 3: dH2^T = W3 dO^T, dZ2 = dH2 gelu'(Z2)
    bf16x4 d2[4][4];
    float gb2[4][4];
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x4 a = load_frag(frag, kTB3 + mt, lane);
        for (int i = 0; i < 4; ++i) gb2[mt][i] = 0.0f;
        for (int st = 0; st < 4; ++st) {
            f32x4 g = mfma(a, dob[st], zero);
            const bf16x4 gz = G2F[(mt * 4 + st) * 64 + lane];
            for (int i = 0; i < 4; ++i) {
                g[i] *= bf2f((unsigned short)gz[i]);
                gb2[mt][i] += g[i];
            }
            d2[mt][st] = pack4(g[0], g[1], g[2], g[3]);
            for (int i = 0; i < 4; ++i) D2T[(mt * 16 + 4 * q + i) * 64 + st * 16 + r] = (unsigned short)d2[mt][st][i];
        }
    }
    // ---- through layer 2: dH1^T = W2 dZ2^T, dZ1 = dH1 gelu'(Z1)
    float gb1[4][4];
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc[4] = {zero, zero, zero, zero};
        for (int kt = 0; kt < 4; ++kt) {
            const bf16x4 a = load_frag(frag, kTB2 + mt * 4 + kt, lane);
            for (int st = 0; st < 4; ++st) acc[st] = mfma(a, d2[kt][st], acc[st]);
        }
        for (int i = 0; i < 4; ++i) gb1[mt][i] = 0.0f;
        for (int st = 0; st < 4; ++st) {
            f32x4 g = acc[st];
            const bf16x4 gz = G1F[(mt * 4 + st) * 64 + lane];
            for (int i = 0; i < 4; ++i) {
                g[i] *= bf2f((unsigned short)gz[i]);
                gb1[mt][i] += g[i];
            }
            const bf16x4 gb = pack4(g[0], g[1], g[2], g[3]);
            for (int i = 0; i < 4; ++i) D1T[(mt * 16 + 4 * q + i) * 64 + st * 16 + r] = (unsigned short)gb[i];
        }
    }
    __syncthreads();
    // ---- weight gradients: contractions over the 64 samples (K dimension)
    for (int mt = 0; mt < 4; ++mt) {               // dW3[hid][o] = sum_s H2[s][hid] dO[s][o]
        f32x4 acc = zero;
        for (int kt = 0; kt < 4; ++kt) acc = mfma(fragT(H2T, mt * 16, kt), fragT(DOT, 0, kt), acc);
        if (r < kOut)
            for (int i = 0; i < 4; ++i) part[kOffW3 + (mt * 16 + 4 * q + i) * kOut + r] = acc[i];
    }
    for (int mt = 0; mt < 4; ++mt)                 // dW2[h1][h2] = sum_s H1[s][h1] dZ2[s][h2]
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = zero;
            for (int kt = 0; kt < 4; ++kt) acc = mfma(fragT(H1T, mt * 16, kt), fragT(D2T, nt * 16, kt), acc);
            for (int i = 0; i < 4; ++i) part[kOffW2 + (mt * 16 + 4 * q + i) * kH + nt * 16 + r] = acc[i];
        }
    for (int nt = 0; nt < 4; ++nt) {               // dW1[f][h] = sum_s X[s][f] dZ1[s][h]
        f32x4 acc = zero;
        for (int kt = 0; kt < 4; ++kt) acc = mfma(fragT(XT, 0, kt), fragT(D1T, nt * 16, kt), acc);
        for (int i = 0; i < 4; ++i) {
            const int f = 4 * q + i;
            if (f < kIn) part[kOffW1 + f * kH + nt * 16 + r] = acc[i];
        }
    }
    // ---- bias gradients: FP32 row sums over the samples (16 lanes of a row group)
    for (int mt = 0; mt < 4; ++mt)
        for (int i = 0; i < 4; ++i) {
            float v1 = gb1[mt][i], v2 = gb2[mt][i];
            for (int w = 1; w < 16; w <<= 1) {
                v1 += __shfl_xor(v1, w);
                v2 += __shfl_xor(v2, w);
            }
            if (r == 0) {
                part[kOffB1 + mt * 16 + 4 * q + i] = v1;
                part[kOffB2 + mt * 16 + 4 * q + i] = v2;
            }
        }
    for (int w = 1; w < 16; w <<= 1) {
        db3[0] += __shfl_xor(db3[0], w);
        db3[1] += __shfl_xor(db3[1], w);
    }
    if (lane == 0) {
        part[kOffB3] = db3[0];
        part[kOffB3 + 1] = db3[1];
    }
    red[lane] = sq;
    __syncthreads();
    if (lane == 0) {
        float t = 0.0f;
        for (int i = 0; i < 64; ++i) t += red[i];
        part[kNPar] = 0.5f * t * inv_n;
    }
}

// Sum the per-workgroup partials in a fixed order.  grad (may be null)
// receives the gradient, loss (may be null) the loss; with adam != 0 the
// bias-corrected Adam step (Kingma & Ba 2015) is applied to theta in place.
__global__ void reduce_adam_kernel(const float *__restrict__ partials, int nblk, float *grad, float *loss,
                                   float *theta, float *m, float *v, int adam, int t, float lr, float b1, float b2,
                                   float eps)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNPar) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += partials[(size_t)b * (kNPar + 1) + p];
    if (p == kNPar) {
        if (loss) *loss = g;
        return;
    }
    if (grad) grad[p] = g;
    if (adam) {
        const float mm = b1 * m[p] + (1.0f - b1) * g;
        const float vv = b2 * v[p] + (1.0f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
        theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

}  // namespace mlp
}  // namespace ppmlr
