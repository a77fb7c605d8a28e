// Finiteness report of a linearization (the device-side info of gnmpc_linearize):
// for the inputs xhat (stages 0..N-1) and uhat and the outputs A, B, c and fnext,
// the number of entries that are NaN or infinite, and the first of them in the
// order (array, element index), mapped back to its stage and node.  Two launches,
// both of fixed shape so that the result does not depend on scheduling: every
// workgroup counts its grid-stride share of each array and writes one partial
// record per array (no atomics, nothing to clear first), then one workgroup sums
// the records in workgroup order and writes the report.
#include <hip/hip_runtime.h>

#include <climits>

#include "plan.hpp"

namespace gnmpc {
namespace {

constexpr int kArrays = 6;           // xhat, uhat, A, B, c, fnext
constexpr int kCheckBlocks = 1024;   // four per CU
constexpr int kCheckThreads = 256;

struct CheckArgs {
  const void* ptr[kArrays];
  long count[kArrays];  // 0 for an absent fnext
  int M, nu, N;
  long nnz;
  const int32_t* erow;  // row node of each pattern entry
  long long* part;      // [kCheckBlocks][kArrays][2]: count, first index (LLONG_MAX if none)
  gnmpc_lin_info* info;
};

template <typename T>
__global__ void __launch_bounds__(kCheckThreads) lin_check_kernel(CheckArgs a) {
  __shared__ long long red_n[kCheckThreads], red_f[kCheckThreads];
  const long stride = (long)gridDim.x * kCheckThreads;
  for (int arr = 0; arr < kArrays; ++arr) {
    const T* v = static_cast<const T*>(a.ptr[arr]);
    long long n = 0, first = LLONG_MAX;
    for (long t = (long)blockIdx.x * kCheckThreads + threadIdx.x; t < a.count[arr]; t += stride) {
      if (!isfinite(v[t])) {
        ++n;
        first = first < t ? first : t;
      }
    }
    red_n[threadIdx.x] = n;
    red_f[threadIdx.x] = first;
    __syncthreads();
    for (int h = kCheckThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        red_n[threadIdx.x] += red_n[threadIdx.x + h];
        red_f[threadIdx.x] = min(red_f[threadIdx.x], red_f[threadIdx.x + h]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      a.part[((size_t)blockIdx.x * kArrays + arr) * 2] = red_n[0];
      a.part[((size_t)blockIdx.x * kArrays + arr) * 2 + 1] = red_f[0];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kCheckBlocks) lin_report_kernel(CheckArgs a) {
  __shared__ long long red_n[kCheckBlocks], red_f[kCheckBlocks];
  __shared__ long long tot[kArrays], fst[kArrays];
  for (int arr = 0; arr < kArrays; ++arr) {
    red_n[threadIdx.x] = a.part[((size_t)threadIdx.x * kArrays + arr) * 2];
    red_f[threadIdx.x] = a.part[((size_t)threadIdx.x * kArrays + arr) * 2 + 1];
    __syncthreads();
    for (int h = kCheckBlocks / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        red_n[threadIdx.x] += red_n[threadIdx.x + h];
        red_f[threadIdx.x] = min(red_f[threadIdx.x], red_f[threadIdx.x + h]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      tot[arr] = red_n[0];
      fst[arr] = red_f[0];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  gnmpc_lin_info r;
  r.status = GNMPC_LIN_FINITE;
  r.first_array = r.first_stage = r.first_node = -1;
  for (int arr = 0; arr < kArrays; ++arr) r.nonfinite[arr] = tot[arr];
  for (int arr = 0; arr < kArrays; ++arr) {
    if (tot[arr] == 0) continue;
    const long long t = fst[arr];
    const long sM = (long)a.M * NBX;
    r.first_array = arr;
    r.status = arr < 2 ? GNMPC_LIN_NONFINITE_INPUT : GNMPC_LIN_NONFINITE_OUTPUT;
    if (arr == 1) {  // uhat [N][nu]
      r.first_stage = (int)(t / a.nu);
    } else if (arr == 2) {  // A [N][nnz][6][6]: the row node of the entry
      r.first_stage = (int)(t / (a.nnz * 36));
      r.first_node = a.erow[(t / 36) % a.nnz];
    } else if (arr == 3) {  // B [N][M][6][nu]
      r.first_stage = (int)(t / (sM * a.nu));
      r.first_node = (int)((t / ((long)NBX * a.nu)) % a.M);
    } else {  // xhat, c, fnext [.][M][6]
      r.first_stage = (int)(t / sM);
      r.first_node = (int)((t / NBX) % a.M);
    }
    break;
  }
  // inputs come first in the order, so a non-finite input decides the status
  // even when an output is non-finite too
  *a.info = r;
}

}  // namespace

size_t lin_check_bytes() { return sizeof(long long) * kCheckBlocks * kArrays * 2; }

gnmpc_status launch_lin_check(gnmpc_plan* p, const void* xhat, const void* uhat, const void* A, const void* B,
                              const void* c, const void* fnext, gnmpc_lin_info* info, hipStream_t s) {
  const int N = p->dims.N, M = p->M, nu = p->dims.nu;
  CheckArgs a;
  const void* ptrs[kArrays] = {xhat, uhat, A, B, c, fnext};
  const long sM = (long)M * NBX;
  const long counts[kArrays] = {N * sM, (long)N * nu, (long)N * p->nnz * 36, N * sM * nu, N * sM,
                                fnext ? N * sM : 0};
  for (int arr = 0; arr < kArrays; ++arr) {
    a.ptr[arr] = ptrs[arr];
    a.count[arr] = counts[arr];
  }
  a.M = M;
  a.nu = nu;
  a.N = N;
  a.nnz = p->nnz;
  a.erow = p->d_erow;
  a.part = static_cast<long long*>(p->d_check);
  a.info = info;
  if (p->dims.dtype == GNMPC_F64)
    lin_check_kernel<double><<<kCheckBlocks, kCheckThreads, 0, s>>>(a);
  else
    lin_check_kernel<float><<<kCheckBlocks, kCheckThreads, 0, s>>>(a);
  lin_report_kernel<<<1, kCheckBlocks, 0, s>>>(a);
  GNMPC_HIP_TRY(p, hipGetLastError());
  return GNMPC_OK;
}

}  // namespace gnmpc
