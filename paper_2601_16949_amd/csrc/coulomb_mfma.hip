// Coulomb pair on the FP32 matrix cores for many slices (a batch of 16 or more right-hand sides):
// with 2R slices the two products are skinny GEMMs, d = B_ov X^T (N_Q x 2R) and J = 2 d^T B_ov
// (2R x ov), and the vector-unit GEMVs that serve a few slices spend most of a step's compute on
// them.  v_mfma_f32_16x16x4f32: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; register t
// of the result is D[4 (l / 16) + t][l % 16].  Operands are staged in LDS with coalesced loads
// (BF16 factors are widened to FP32 on the way).  Each output element is a fixed-order sum whose
// order does not depend on the slice count, so a batch and one of its RHS alone give the same d
// and J bitwise.
#include "common.h"

namespace rttda {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float ld(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld(const __hip_bfloat16 *p, size_t i) { return __bfloat162float(p[i]); }

constexpr int CM_QT = 64;   // Q rows per workgroup of the first product (16 per wave)
constexpr int CM_ST = 128;  // slices per workgroup (8 blocks of 16)
constexpr int CM_KT = 32;   // K values staged per LDS round
constexpr int CM_LD = CM_KT + 1;

// dpart[chunk][q][s] = sum over the chunk's ia of B[q][ia] X[s][ia]; grid (Q blocks, slice blocks, chunks)
template <typename TB>
__global__ __launch_bounds__(256) void k_coul1_mfma(const TB *__restrict__ B, const float *__restrict__ X, int nq,
                                                    int ov, int ns, int echunk, float *__restrict__ dpart) {
  __shared__ float As[CM_QT][CM_LD];
  __shared__ float Bs[CM_ST][CM_LD];
  const int q0 = blockIdx.x * CM_QT, s0 = blockIdx.y * CM_ST;
  const int e0 = blockIdx.z * echunk, e1 = min(ov, e0 + echunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f4v acc[CM_ST / 16];
#pragma unroll
  for (int j = 0; j < CM_ST / 16; ++j) acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int e = e0; e < e1; e += CM_KT) {
    __syncthreads();  // the previous round's operands have been read
    for (int t = tid; t < CM_QT * CM_KT; t += 256) {
      const int r = t / CM_KT, k = t % CM_KT;
      const int q = q0 + r, ia = e + k;
      As[r][k] = (q < nq && ia < e1) ? ld(B, (size_t)q * ov + ia) : 0.f;
    }
    for (int t = tid; t < CM_ST * CM_KT; t += 256) {
      const int r = t / CM_KT, k = t % CM_KT;
      const int sl = s0 + r, ia = e + k;
      Bs[r][k] = (sl < ns && ia < e1) ? X[(size_t)sl * ov + ia] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < CM_KT / 4; ++kk) {
      const float a = As[16 * wave + li][4 * kk + lk];
#pragma unroll
      for (int j = 0; j < CM_ST / 16; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Bs[16 * j + li][4 * kk + lk], acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < CM_ST / 16; ++j)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = q0 + 16 * wave + 4 * lk + t, sl = s0 + 16 * j + li;
      if (q < nq && sl < ns) dpart[((size_t)blockIdx.z * nq + q) * ns + sl] = acc[j][t];
    }
}

__global__ void k_dsum_m(float *__restrict__ dpart, int n, int nes) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float d = dpart[e];
    for (int k = 1; k < nes; ++k) d += dpart[(size_t)k * n + e];
    dpart[e] = d;
  }
}

constexpr int CM_IT = 64;  // ia columns per workgroup of the second product (16 per wave)

// P[split][s][ia] = 2 sum_{Q in split} d[Q][s] B[Q][ia]; grid (ia blocks, slice blocks, splits)
template <typename TB>
__global__ __launch_bounds__(256) void k_coul2_mfma(const TB *__restrict__ B, const float *__restrict__ d, int nq,
                                                    int ov, int ns, int nsplit, float *__restrict__ P) {
  __shared__ float Ds[CM_KT][CM_ST + 1];  // [Q][s]
  __shared__ float Bs[CM_KT][CM_IT + 1];  // [Q][ia]
  const int e0 = blockIdx.x * CM_IT, s0 = blockIdx.y * CM_ST, sp = blockIdx.z;
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f4v acc[CM_ST / 16];
#pragma unroll
  for (int j = 0; j < CM_ST / 16; ++j) acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int q = qa; q < qb; q += CM_KT) {
    __syncthreads();
    for (int t = tid; t < CM_KT * CM_ST; t += 256) {
      const int k = t / CM_ST, c = t % CM_ST;
      const int qq = q + k, sl = s0 + c;
      Ds[k][c] = (qq < qb && sl < ns) ? d[(size_t)qq * ns + sl] : 0.f;
    }
    for (int t = tid; t < CM_KT * CM_IT; t += 256) {
      const int k = t / CM_IT, c = t % CM_IT;
      const int qq = q + k, ia = e0 + c;
      Bs[k][c] = (qq < qb && ia < ov) ? ld(B, (size_t)qq * ov + ia) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < CM_KT / 4; ++kk) {
      const float b = Bs[4 * kk + lk][16 * wave + li];
#pragma unroll
      for (int j = 0; j < CM_ST / 16; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ds[4 * kk + lk][16 * j + li], b, acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < CM_ST / 16; ++j)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int sl = s0 + 16 * j + 4 * lk + t, ia = e0 + 16 * wave + li;
      if (sl < ns && ia < ov) P[((size_t)sp * ns + sl) * ov + ia] = 2.f * acc[j][t];
    }
}

}  // namespace

int coulomb_mfma_chunks(int nq, int ov) {
  // independent of the slice count (a batch and one of its RHS alone sum d the same way): about
  // 256 workgroups for the first product, at most GEMV1_CHUNKS_MAX chunks of at least 128 ia
  const int qblocks = (nq + CM_QT - 1) / CM_QT;
  const int want = (256 + qblocks - 1) / qblocks;
  return std::max(1, std::min({want, GEMV1_CHUNKS_MAX, std::max(1, ov / 128)}));
}

hipError_t launch_coulomb_mfma(hipStream_t s, int b_dtype, const void *B, const float *X, int nq, int ov, int ns,
                               int nes, int nsplit, float *dpart, float *P) {
  const int echunk = ((ov + nes - 1) / nes + CM_KT - 1) / CM_KT * CM_KT;
  const int nch = (ov + echunk - 1) / echunk;
  const dim3 g1((nq + CM_QT - 1) / CM_QT, (ns + CM_ST - 1) / CM_ST, nch);
  const dim3 g2((ov + CM_IT - 1) / CM_IT, (ns + CM_ST - 1) / CM_ST, nsplit);
  if (b_dtype == RTTDA_BF16) {
    const __hip_bfloat16 *Bb = static_cast<const __hip_bfloat16 *>(B);
    hipLaunchKernelGGL(k_coul1_mfma<__hip_bfloat16>, g1, dim3(256), 0, s, Bb, X, nq, ov, ns, echunk, dpart);
    if (nch > 1) hipLaunchKernelGGL(k_dsum_m, dim3(std::max(1, std::min(1024, (nq * ns + 255) / 256))), dim3(256), 0, s,
                                    dpart, nq * ns, nch);
    hipLaunchKernelGGL(k_coul2_mfma<__hip_bfloat16>, g2, dim3(256), 0, s, Bb, dpart, nq, ov, ns, nsplit, P);
  } else {
    const float *Bf = static_cast<const float *>(B);
    hipLaunchKernelGGL(k_coul1_mfma<float>, g1, dim3(256), 0, s, Bf, X, nq, ov, ns, echunk, dpart);
    if (nch > 1) hipLaunchKernelGGL(k_dsum_m, dim3(std::max(1, std::min(1024, (nq * ns + 255) / 256))), dim3(256), 0, s,
                                    dpart, nq * ns, nch);
    hipLaunchKernelGGL(k_coul2_mfma<float>, g2, dim3(256), 0, s, Bf, dpart, nq, ov, ns, nsplit, P);
  }
  return hipGetLastError();
}

}  // namespace rttda
