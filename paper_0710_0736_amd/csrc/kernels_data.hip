// kernels_data.hip -- image data on refined lattices, the consistent-mass and
// by-simplex views of the image, and the colour-space pre-pass.  Each is one pass over the data
// (HBM bound).
#include <algorithm>

#include "acseg_internal.h"

namespace acseg {

namespace {

constexpr int kRowBlocks = 4096;  // grid-stride over rows: enough workgroups to fill the chip

// Piecewise-constant injection: row Y of plane c of the refined lattice copies
// pixel row Y >> r, each pixel value repeated over the 2^r nodes it owns along
// x (the last pixel owns one node).  One workgroup per row (grid-stride),
// coalesced writes; the pixel row is read from cache 2^r times.
__global__ __launch_bounds__(kBlock) void k_refine(const float* __restrict__ src, float* __restrict__ dst,
                                                   int W, int H, int r, int Wf, int Hf, int planes) {
    const int64_t n = (int64_t)W * H, nf = (int64_t)Wf * Hf;
    const int64_t rows = (int64_t)Hf * planes;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int c = (int)(row / Hf), Y = (int)(row - (int64_t)c * Hf);
        const float* s = src + c * n + (int64_t)(Y >> r) * W;
        float* d = dst + c * nf + (int64_t)Y * Wf;
        for (int X = threadIdx.x; X < Wf; X += kBlock) d[X] = s[X >> r];
    }
}

// The pixel nodes of a refined field: dst[c][y][x] = src[c][y 2^r][x 2^r].
__global__ __launch_bounds__(kBlock) void k_sample(const float* __restrict__ src, float* __restrict__ dst,
                                                   int W, int H, int r, int Wf, int Hf, int planes) {
    const int64_t n = (int64_t)W * H, nf = (int64_t)Wf * Hf;
    const int64_t rows = (int64_t)H * planes;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int c = (int)(row / H), y = (int)(row - (int64_t)c * H);
        const float* s = src + c * nf + ((int64_t)y << r) * Wf;
        float* d = dst + c * n + (int64_t)y * W;
        for (int x = threadIdx.x; x < W; x += kBlock) d[x] = s[(int64_t)x << r];
    }
}

// sRGB (IEC 61966-2-1) to CIE 1976 L*a*b*, divided by 100.
//   linear c = v / 12.92 for v <= 0.04045, else ((v + 0.055) / 1.055)^2.4;
//   (X, Y, Z) = M (r, g, b) with the sRGB primaries' matrix M (D65);
//   f(t) = t^(1/3) for t > (6/29)^3, else t / (3 (6/29)^2) + 4/29;
//   L* = 116 f(Y/Yw) - 16, a* = 500 (f(X/Xw) - f(Y/Yw)), b* = 200 (f(Y/Yw) - f(Z/Zw)),
// with (Xw, Yw, Zw) = M (1, 1, 1), the row sums of M.
__device__ __forceinline__ float srgb_linear(float v) {
    return v <= 0.04045f ? v * (1.f / 12.92f) : powf((v + 0.055f) * (1.f / 1.055f), 2.4f);
}
__device__ __forceinline__ float lab_f(float t) {
    constexpr float d = 6.f / 29.f;
    return t > d * d * d ? cbrtf(t) : t * (1.f / (3.f * d * d)) + 4.f / 29.f;
}

__global__ __launch_bounds__(kBlock) void k_lab(const float* __restrict__ rgb, float* __restrict__ dst,
                                                int64_t count, int ab_only) {
    constexpr float m00 = 0.4124f, m01 = 0.3576f, m02 = 0.1805f;
    constexpr float m10 = 0.2126f, m11 = 0.7152f, m12 = 0.0722f;
    constexpr float m20 = 0.0193f, m21 = 0.1192f, m22 = 0.9505f;
    constexpr float xw = m00 + m01 + m02, yw = m10 + m11 + m12, zw = m20 + m21 + m22;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < count; p += (int64_t)gridDim.x * kBlock) {
        const float r = srgb_linear(rgb[p]), g = srgb_linear(rgb[count + p]), b = srgb_linear(rgb[2 * count + p]);
        const float fx = lab_f((m00 * r + m01 * g + m02 * b) / xw);
        const float fy = lab_f((m10 * r + m11 * g + m12 * b) / yw);
        const float fz = lab_f((m20 * r + m21 * g + m22 * b) / zw);
        const float L = 1.16f * fy - 0.16f, A = 5.f * (fx - fy), B = 2.f * (fy - fz);
        if (ab_only) {
            dst[p] = A;
            dst[count + p] = B;
        } else {
            dst[p] = L;
            dst[count + p] = A;
            dst[2 * count + p] = B;
        }
    }
}

// The image as the consistent P1 mass matrix sees it: (M I)_p / m_p, every
// lattice cell split along its (x,y)-(x+1,y+1) diagonal.  A triangle T at node
// p with other vertices a, b adds |T|/12 (2 I_p + I_a + I_b) to (M I)_p and
// |T|/3 to the lumped mass m_p, so (M I)_p / m_p is the sum over the n_T
// triangles at p of (2 I_p + I_a + I_b), divided by 4 n_T (6 triangles inside;
// fewer on the boundary, at least one).
// SIMPLEX: projection by simplex instead.  Each triangle carries one value, the
// mean (I_p + I_a + I_b) / 3 of its vertices (its integral over |T|), and adds
// |T|/3 of it to node p's load, so the nodal value is the sum over the n_T
// triangles of (I_p + I_a + I_b), divided by 3 n_T.  One workgroup per row.
template <bool SIMPLEX>
__global__ __launch_bounds__(kBlock) void k_mass_avg(const float* __restrict__ src, float* __restrict__ dst,
                                                     int W, int H, int planes) {
    const int64_t n = (int64_t)W * H;
    const int64_t rows = (int64_t)H * planes;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int c = (int)(row / H), y = (int)(row - (int64_t)c * H);
        const float* s = src + c * n;
        float* d = dst + c * n + (int64_t)y * W;
        const float* r0 = s + (int64_t)y * W;            // row y
        const float* rd = y > 0 ? r0 - W : r0;           // row y - 1 (read only when it exists)
        const float* ru = y < H - 1 ? r0 + W : r0;       // row y + 1
        for (int x = threadIdx.x; x < W; x += kBlock) {
            const bool L = x > 0, R = x < W - 1, D = y > 0, U = y < H - 1;
            const float ip2 = SIMPLEX ? r0[x] : 2.f * r0[x];
            float acc = 0.f;
            int nt = 0;
            if (L && D) {  // cell (x-1, y-1): both triangles have p as their (x+1, y+1) corner
                acc += (ip2 + rd[x - 1] + rd[x]) + (ip2 + rd[x - 1] + r0[x - 1]);
                nt += 2;
            }
            if (R && D) {  // cell (x, y-1): triangle (x, y-1), (x, y), (x+1, y)
                acc += ip2 + rd[x] + r0[x + 1];
                nt += 1;
            }
            if (L && U) {  // cell (x-1, y): triangle (x-1, y), (x, y), (x, y+1)
                acc += ip2 + r0[x - 1] + ru[x];
                nt += 1;
            }
            if (R && U) {  // cell (x, y): both triangles have p as their (x, y) corner
                acc += (ip2 + r0[x + 1] + ru[x + 1]) + (ip2 + ru[x] + ru[x + 1]);
                nt += 2;
            }
            d[x] = acc / (float)((SIMPLEX ? 3 : 4) * nt);
        }
    }
}

int row_blocks(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(rows, kRowBlocks)); }

}  // namespace

hipError_t launch_refine(int planes, int W, int H, int r, const float* src, float* dst, hipStream_t s) {
    const int Wf = ((W - 1) << r) + 1, Hf = ((H - 1) << r) + 1;
    hipLaunchKernelGGL(k_refine, dim3(row_blocks((int64_t)Hf * planes)), dim3(kBlock), 0, s, src, dst, W, H, r,
                       Wf, Hf, planes);
    return hipGetLastError();
}

hipError_t launch_sample(int planes, int W, int H, int r, const float* src, float* dst, hipStream_t s) {
    const int Wf = ((W - 1) << r) + 1, Hf = ((H - 1) << r) + 1;
    hipLaunchKernelGGL(k_sample, dim3(row_blocks((int64_t)H * planes)), dim3(kBlock), 0, s, src, dst, W, H, r,
                       Wf, Hf, planes);
    return hipGetLastError();
}

hipError_t launch_mass_avg(int planes, int W, int H, const float* src, float* dst, int simplex, hipStream_t s) {
    if (simplex)
        hipLaunchKernelGGL(k_mass_avg<true>, dim3(row_blocks((int64_t)H * planes)), dim3(kBlock), 0, s, src, dst,
                           W, H, planes);
    else
        hipLaunchKernelGGL(k_mass_avg<false>, dim3(row_blocks((int64_t)H * planes)), dim3(kBlock), 0, s, src, dst,
                           W, H, planes);
    return hipGetLastError();
}

hipError_t launch_lab(int ab_only, int64_t count, const float* rgb, float* dst, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((count + kBlock - 1) / kBlock, 8192));
    hipLaunchKernelGGL(k_lab, dim3(blocks), dim3(kBlock), 0, s, rgb, dst, count, ab_only);
    return hipGetLastError();
}

}  // namespace acseg
