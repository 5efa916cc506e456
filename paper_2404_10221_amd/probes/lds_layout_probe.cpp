// LDS bank-conflict probe for gfx950 (not part of the library).  Each kernel
// makes one 16-byte-per-lane LDS access pattern 16 x 8 times per workgroup; run
// it under rocprofv3 with SQ_LDS_IDX_ACTIVE and SQ_LDS_BANK_CONFLICT to read the
// conflict cycles of each pattern.  Patterns: unit-stride reads and writes with
// lane groups offset against 16-byte slots (how the hardware groups lanes), and
// the Stockham accesses of a 2048-point radix-8 plan (256 threads, 8 elements
// each) under three sequence layouts: one pad slot per 256 bytes (padded), no
// padding (plain), and an XOR of (i >> 3) & 7 into the slot (swizzled).
// Build: hipcc --offload-arch=gfx950 -O3 -o lds_layout_probe lds_layout_probe.cpp
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

struct c2 {
  double x, y;
};

// lane-group offsets: slot of lane t (64 lanes, one wavefront window of 256 slots)
__device__ __forceinline__ int lane_slot(int P, int t) {
  switch (P) {
    case 0: return t;                 // unit stride
    case 1: return t + (t / 16);      // +1 slot per 16 lanes
    case 2: return t + (t / 8);       // +1 slot per 8 lanes
    case 3: return t + (t / 32);      // +1 slot per 32 lanes
    case 4: return t + 1;             // whole wavefront shifted by 16 bytes
    case 5: return t ^ 1;             // pairs swapped inside a row
    case 6: return t * 2;             // stride 2 slots
    default: return t + 16 * (t / 16);  // 16-lane groups 512 bytes apart
  }
}

template <int P, bool WR>
__global__ void __launch_bounds__(256) k_lanes(const double* __restrict__ in, double* __restrict__ out) {
  __shared__ c2 s[1024];
  const int t = threadIdx.x;
  const double v = in[blockIdx.x * 256 + t];
  for (int i = t; i < 1024; i += 256) s[i] = c2{v, v};
  __syncthreads();
  double acc = 0.0;
  const int sl = (t >> 6) * 256 + lane_slot(P, t & 63);
  for (int rep = 0; rep < 64; ++rep) {
    if (WR) {
      s[sl] = c2{v + rep, v};
    } else {
      const c2 q = s[sl];
      acc += q.x * q.y;
    }
    __builtin_amdgcn_s_barrier();
  }
  __syncthreads();
  out[blockIdx.x * 256 + t] = acc + s[t].x;
}

template <int LAY>
__device__ __forceinline__ int seq_slot(int i) {
  if (LAY == 0) return i + (i >> 4);          // padded
  if (LAY == 1) return i;                     // plain
  return i ^ ((i >> 3) & 7);                  // swizzled
}

// element of access r (of 8) of thread t in each Stockham pattern
template <int PAT>
__device__ __forceinline__ int stage_elem(int t, int r, bool& wr) {
  wr = true;
  switch (PAT) {
    case 0: wr = false; return t + r * 256;                                    // stage read x[j + r L/R]
    case 1: return 8 * t + r;                                                  // stage-0 write (stride 8)
    case 2: return (t / 8) * 64 + t % 8 + 8 * r;                               // stage-1 write
    case 3: { const int j = t + 256 * (r >> 2); return j + 512 * (r & 3); }    // last (radix-4) write
    default: wr = false; return r < 4 ? t + 256 * r : (8 - r) * 256 - t;       // mirrored read (odd extension)
  }
}

template <int LAY, int PAT>
__global__ void __launch_bounds__(256) k_stage(const double* __restrict__ in, double* __restrict__ out) {
  __shared__ c2 s[2304];
  const int t = threadIdx.x;
  const double v = in[blockIdx.x * 256 + t];
  for (int i = t; i < 2304; i += 256) s[i] = c2{v, v};
  __syncthreads();
  double acc = 0.0;
  for (int rep = 0; rep < 16; ++rep) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      bool wr;
      const int p = seq_slot<LAY>(stage_elem<PAT>(t, r, wr));
      if (wr) {
        s[p] = c2{v + r, v - rep};
      } else {
        const c2 q = s[p];
        acc += q.x * q.y;
      }
    }
    __syncthreads();
  }
  out[blockIdx.x * 256 + t] = acc + s[t].x;
}

template <int P>
static void lanes(const double* in, double* out) {
  hipLaunchKernelGGL((k_lanes<P, false>), dim3(2048), dim3(256), 0, 0, in, out);
  hipLaunchKernelGGL((k_lanes<P, true>), dim3(2048), dim3(256), 0, 0, in, out);
}
template <int LAY>
static void stages(const double* in, double* out) {
  hipLaunchKernelGGL((k_stage<LAY, 0>), dim3(1024), dim3(256), 0, 0, in, out);
  hipLaunchKernelGGL((k_stage<LAY, 1>), dim3(1024), dim3(256), 0, 0, in, out);
  hipLaunchKernelGGL((k_stage<LAY, 2>), dim3(1024), dim3(256), 0, 0, in, out);
  hipLaunchKernelGGL((k_stage<LAY, 3>), dim3(1024), dim3(256), 0, 0, in, out);
  hipLaunchKernelGGL((k_stage<LAY, 4>), dim3(1024), dim3(256), 0, 0, in, out);
}

int main() {
  const int n = 2048 * 256;
  double *in = nullptr, *out = nullptr;
  if (hipMalloc(&in, n * sizeof(double)) != hipSuccess || hipMalloc(&out, n * sizeof(double)) != hipSuccess) return 1;
  std::vector<double> h(n, 1.0);
  if (hipMemcpy(in, h.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;
  lanes<0>(in, out); lanes<1>(in, out); lanes<2>(in, out); lanes<3>(in, out);
  lanes<4>(in, out); lanes<5>(in, out); lanes<6>(in, out); lanes<7>(in, out);
  stages<0>(in, out); stages<1>(in, out); stages<2>(in, out);
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  if (hipMemcpy(h.data(), out, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
  printf("lds layout probe done %g\n", h[0]);
  (void)hipFree(in);
  (void)hipFree(out);
  return 0;
}
