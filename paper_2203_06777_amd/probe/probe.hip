// Measurement probes for the benchmark (libdwf_probe.so): not part of the operator library.
//
// probe_stream_rows: the compulsory traffic of one checkerboard hopping apply in the row
//   kernel's shape and nothing else: workgroup q reads one links block (vl 16-byte vectors) and
//   one input row (vx vectors) and writes one output row (vx vectors, non-temporal stores).  Its
//   time is the bandwidth a kernel moving exactly those bytes reaches on this chip.
// probe_dhop_pattern: the memory accesses of the FP32 row kernel at L^3 rows of 256 lanes (L0h = 16,
//   Ls = 16) and nothing else: same XCD remap and (ty, tz, tt) row order, the links block and the
//   own row read once per workgroup, each lane's six y/z/t neighbour spinors (6 vectors each) read
//   (or, with neighbours = 0, not), the output row written with non-temporal stores (or, with
//   stores = 0, not); the values only feed an xor.
// probe_read: reads n 16-byte vectors over and over with a grid-stride loop (footprints that fit
//   the L2, the Infinity Cache or neither).
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

__device__ inline unsigned xcd_block(unsigned b, unsigned nb) {  // consecutive blocks per XCD
    const unsigned q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

template <int NBR, int STORE>
__global__ void __launch_bounds__(256) k_dhop_pattern(u32x4 *__restrict__ out, const u32x4 *__restrict__ in,
                                                      const u32x4 *__restrict__ lk, unsigned L, unsigned ty,
                                                      unsigned tz, unsigned tt) {
    const unsigned q = xcd_block(blockIdx.x, gridDim.x);
    const unsigned per = ty * tz * tt;
    const unsigned T = q / per, w = q % per;
    const unsigned ly = w % ty, lz = (w / ty) % tz, lt = w / (ty * tz);
    const unsigned ntt = L / tt, nty = L / ty;
    const unsigned Tt = T % ntt, Ty = (T / ntt) % nty, Tz = T / (ntt * nty);
    const unsigned y = Ty * ty + ly, z = Tz * tz + lz, t3 = Tt * tt + lt;
    const unsigned row = y + L * (z + L * t3);
    const int t = threadIdx.x, xh = t >> 4, s = t & 15;
    constexpr unsigned VX = 1536, VL = 576;  // 16-byte vectors per row: input (16 sites x 16 s x 96 B), links
    const u32x4 *Lr = lk + (size_t)row * VL;
    const u32x4 *I = in + (size_t)row * VX;
    u32x4 acc = Lr[t] ^ Lr[256 + t];
    if (t < 64) acc ^= Lr[512 + t];
#pragma unroll
    for (int u = 0; u < 6; ++u) acc ^= I[u * 256 + t];
    if (NBR) {
        const unsigned nb[6] = {((y + 1) % L) + L * (z + L * t3), y + L * (((z + 1) % L) + L * t3),
                                y + L * (z + L * ((t3 + 1) % L)), ((y + L - 1) % L) + L * (z + L * t3),
                                y + L * (((z + L - 1) % L) + L * t3), y + L * (z + L * ((t3 + L - 1) % L))};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const u32x4 *N = in + (size_t)nb[k] * VX + xh * 96 + s;
#pragma unroll
            for (int g = 0; g < 6; ++g) acc ^= N[g * 16];
        }
    }
    u32x4 *O = out + (size_t)row * VX;
    if (STORE) {
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            u32x4 v = acc;
            v.x += u;
            __builtin_nontemporal_store(v, O + u * 256 + t);
        }
    } else if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u) {
        O[t] = acc;  // keeps the loads; practically never taken
    }
}

__global__ void k_read(const u32x4 *__restrict__ in, u32x4 *sink, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t st = (size_t)gridDim.x * blockDim.x;
    u32x4 acc = {0, 0, 0, 0};
    for (; i < n; i += st) acc ^= in[i];
    if (acc.x == 0x12345678u && acc.y == 0x9abcdef0u) sink[0] = acc;
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

// L^3 rows; in and out hold L^3 * 1536 vectors, links L^3 * 576; ty, tz, tt divide L.
int probe_dhop_pattern(void *out, const void *in, const void *links, unsigned L, unsigned ty, unsigned tz, unsigned tt,
                       int neighbours, int stores, void *stream) {
    if (!out || !in || !links || L == 0 || !ty || !tz || !tt || L % ty || L % tz || L % tt) return -1;
    const hipStream_t st = (hipStream_t)stream;
    const unsigned nrows = L * L * L;
    u32x4 *o = (u32x4 *)out;
    const u32x4 *i = (const u32x4 *)in, *l = (const u32x4 *)links;
    if (neighbours && stores) hipLaunchKernelGGL((k_dhop_pattern<1, 1>), dim3(nrows), dim3(256), 0, st, o, i, l, L, ty, tz, tt);
    else if (neighbours) hipLaunchKernelGGL((k_dhop_pattern<1, 0>), dim3(nrows), dim3(256), 0, st, o, i, l, L, ty, tz, tt);
    else if (stores) hipLaunchKernelGGL((k_dhop_pattern<0, 1>), dim3(nrows), dim3(256), 0, st, o, i, l, L, ty, tz, tt);
    else hipLaunchKernelGGL((k_dhop_pattern<0, 0>), dim3(nrows), dim3(256), 0, st, o, i, l, L, ty, tz, tt);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int probe_read(const void *in, void *sink, size_t nvec, void *stream) {
    if (!in || !sink || nvec == 0) return -1;
    hipLaunchKernelGGL(k_read, dim3(8192), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)in, (u32x4 *)sink, nvec);
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
