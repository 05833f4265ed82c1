// Measurement probes for the benchmark (libdwf_probe.so): not part of the operator library.
//
// probe_stream_rows: the compulsory traffic of one checkerboard hopping apply in the row
//   kernel's shape and nothing else: workgroup q reads one links block (vl 16-byte vectors) and
//   one input row (vx vectors) and writes one output row (vx vectors, non-temporal stores).  Its
//   time is the bandwidth a kernel moving exactly those bytes reaches on this chip.
// probe_link_mult: the SU(3) link multiply as a (6 x 6 real) x (6 x N real) product, three ways:
//   mode 0  vector ALU: lane j holds column j (6 reals) and multiplies it by the matrix (36 FMAs);
//   mode 1  matrix cores, operands already in the MFMA layout: A = the matrix padded to 16 x 8,
//           B = 8 x 16 columns, two v_mfma_f32_16x16x4f32 per product (K = 8 in two steps of 4);
//   mode 2  matrix cores with the columns held one per lane as in the stencil: lane shuffles move
//           them into the B layout and the 6 x 16 result back.
//   Each wave repeats the product reps times on its own columns (the result feeds the next round);
//   out receives the final columns.  One round of mode 1 or 2 is checked against a CPU product.
#include <hip/hip_runtime.h>

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_rows(u32x4 *__restrict__ out, const u32x4 *__restrict__ in,
                                                     const u32x4 *__restrict__ lk, unsigned vx, unsigned vl) {
    const unsigned q = blockIdx.x;
    const u32x4 *L = lk + (size_t)q * vl;
    const u32x4 *I = in + (size_t)q * vx;
    u32x4 *O = out + (size_t)q * vx;
    u32x4 m = {0, 0, 0, 0};
    for (unsigned v = threadIdx.x; v < vl; v += blockDim.x) m ^= L[v];
    for (unsigned v = threadIdx.x; v < vx; v += blockDim.x) {
        u32x4 w = I[v];
        w.x ^= m.x ^ m.y ^ m.z ^ m.w;
        __builtin_nontemporal_store(w, O + v);
    }
}

// mat: 36 floats (row-major 6 x 6), the same for every wave; cols: per wave 64 columns of 6 floats
// (column-major: cols[(wave * 64 + j) * 6 + k]).
__global__ void __launch_bounds__(256) k_mult_valu(float *out, const float *mat, const float *cols, int reps) {
    const int lane = threadIdx.x & 63;
    const long col = (long)blockIdx.x * 256 + threadIdx.x;
    float m[36], x[6];
#pragma unroll
    for (int k = 0; k < 36; ++k) m[k] = mat[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = cols[col * 6 + k];
    (void)lane;
    for (int r = 0; r < reps; ++r) {
        float y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            float acc = m[i * 6] * x[0];
#pragma unroll
            for (int k = 1; k < 6; ++k) acc = __builtin_fmaf(m[i * 6 + k], x[k], acc);
            y[i] = acc;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) x[k] = y[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) out[col * 6 + k] = x[k];
}

// One wave per 16 columns (wave w of the grid: columns w*16 .. w*16+15).
// v_mfma_f32_16x16x4f32 layout: A[i][k] in lane i + 16 k; B[k][j] in lane j + 16 k; C[i][j] in
// lane j + 16 (i / 4), element i % 4.
template <int SHUF>
__global__ void __launch_bounds__(256) k_mult_mfma(float *out, const float *mat, const float *cols, int reps) {
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    // A, K steps 0 (k = kq) and 1 (k = 4 + kq): rows i16 < 6, columns k < 6
    const float a0 = (i16 < 6) ? mat[i16 * 6 + kq] : 0.f;
    const float a1 = (i16 < 6 && 4 + kq < 6) ? mat[i16 * 6 + 4 + kq] : 0.f;
    const float *cw = cols + wave * 16 * 6;
    f32x4 c = {0, 0, 0, 0};
    float b0, b1;
    float xl[6];  // SHUF: lane j < 16 holds column j, as the stencil's lanes hold their half spinors
    if (SHUF) {
#pragma unroll
        for (int k = 0; k < 6; ++k) xl[k] = i16 == lane ? cw[i16 * 6 + k] : 0.f;
    }
    b0 = cw[i16 * 6 + kq];
    b1 = 4 + kq < 6 ? cw[i16 * 6 + 4 + kq] : 0.f;
    for (int r = 0; r < reps; ++r) {
        if (SHUF) {
            // B[k][j] = column j element k, held by lane j: read register k of lane j
            float g[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) g[k] = __shfl(xl[k], i16, 64);
            b0 = kq == 0 ? g[0] : kq == 1 ? g[1] : kq == 2 ? g[2] : g[3];
            b1 = kq == 0 ? g[4] : kq == 1 ? g[5] : 0.f;
        }
        c = f32x4{0, 0, 0, 0};
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, c, 0, 0, 0);
        if (SHUF) {
            // back to one column per lane: y_j[i] = C[i][j] in lane j + 16 (i / 4), element i % 4
#pragma unroll
            for (int i = 0; i < 6; ++i) xl[i] = __shfl(c[i & 3], i16 + 16 * (i >> 2), 64);
        } else {
            // operands stay in the MFMA layout; the result feeds the next round in place
            b0 = c[0];
            b1 = c[1];
        }
    }
    // lane j + 16 q holds C[4 q + e][j]: rows < 6 are the product's rows
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * kq + e;
        if (row < 6) out[(wave * 16 + i16) * 6 + row] = c[e];
    }
}

extern "C" {

int probe_stream_rows(void *out, const void *in, const void *links, unsigned nrows, unsigned vx, unsigned vl,
                      void *stream) {
    if (!out || !in || !links || nrows == 0) return -1;
    hipLaunchKernelGGL(k_stream_rows, dim3(nrows), dim3(256), 0, (hipStream_t)stream, (u32x4 *)out,
                       (const u32x4 *)in, (const u32x4 *)links, vx, vl);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// nwg workgroups of 256 lanes; mode 0: 256 columns per workgroup, modes 1-2: 64 (16 per wave).
int probe_link_mult(float *out, const float *mat, const float *cols, int mode, int nwg, int reps, void *stream) {
    if (!out || !mat || !cols || nwg <= 0 || reps < 1 || mode < 0 || mode > 2) return -1;
    const hipStream_t st = (hipStream_t)stream;
    if (mode == 0) hipLaunchKernelGGL(k_mult_valu, dim3(nwg), dim3(256), 0, st, out, mat, cols, reps);
    else if (mode == 1) hipLaunchKernelGGL(k_mult_mfma<0>, dim3(nwg), dim3(256), 0, st, out, mat, cols, reps);
    else hipLaunchKernelGGL(k_mult_mfma<1>, dim3(nwg), dim3(256), 0, st, out, mat, cols, reps);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
