// GMPEA generation kernels for 4 <= m <= 8 objectives (the many-objective
// generalisation): the device code of gmpea_device.hpp instantiated per m, with
// F/CV records and reference-vector rows of rec_quads(m) float4. Kept apart from
// the m <= 3 kernels so that those keep their register budget: in a batched
// launch one kernel serves every instance of its list, and its register count
// is the largest over the m values it dispatches.
//
// Per m the generation is the m <= 3 one: k_vary (mating, variation,
// evaluation, ideal point), k_op1, then k_select (decisions and locations).
// Register use grows with m through the records a k_select lane keeps (its
// parent, weight, best candidate and four candidates in flight); the evaluation
// keeps the leading variables (the m - 1 angles) of its group's first chunks.
#include <type_traits>

#include "gmpea_device.hpp"

// Built with -ffp-contract=off like the m <= 3 kernels: every fused multiply-add
// is an explicit fmaf, so plain and batched launches round identically.

namespace gmpea {

template <class F>
static void with_lanes(const DevState &st, F &&f) {
  switch (vary_lanes_of(st)) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

template <class F>
static void with_wide_m(int m, F &&f) {
  switch (m) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}

// Batched phases over instances with m > 3 (the sphere family).
template <int M>
__device__ __forceinline__ void vary_batch_m(const DevState &st, int L) {
  vary_any_lanes<M, 1>(st, L);
}

__global__ __launch_bounds__(kBlock) void k_vary_batch_w(const DevState *__restrict__ S,
                                                        const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  switch (st.m) {
    case 4: vary_batch_m<4>(st, wi.y); break;
    case 5: vary_batch_m<5>(st, wi.y); break;
    case 6: vary_batch_m<6>(st, wi.y); break;
    case 7: vary_batch_m<7>(st, wi.y); break;
    default: vary_batch_m<8>(st, wi.y); break;
  }
}

__global__ __launch_bounds__(kBlock) void k_tvary_batch_w(const DevState *__restrict__ S,
                                                         const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  switch (st.m) {
    case 4: tvary_body<4, 1>(st, wi.y, vary_grid(st)); break;
    case 5: tvary_body<5, 1>(st, wi.y, vary_grid(st)); break;
    case 6: tvary_body<6, 1>(st, wi.y, vary_grid(st)); break;
    case 7: tvary_body<7, 1>(st, wi.y, vary_grid(st)); break;
    default: tvary_body<8, 1>(st, wi.y, vary_grid(st)); break;
  }
}

__global__ __launch_bounds__(kBlock) void k_op1_batch_w(const DevState *__restrict__ S,
                                                       const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  switch (st.m) {
    case 4: op1_body<4>(st, wi.y); break;
    case 5: op1_body<5>(st, wi.y); break;
    case 6: op1_body<6>(st, wi.y); break;
    case 7: op1_body<7>(st, wi.y); break;
    default: op1_body<8>(st, wi.y); break;
  }
}

__global__ __launch_bounds__(kBlock) void k_select_batch_w(const DevState *__restrict__ S,
                                                          const int2 *__restrict__ work) {
  const int2 wi = work[blockIdx.x];
  if (wi.x < 0) return;
  const DevState &st = S[wi.x];
  switch (st.m) {
    case 4: select_body<4>(st, wi.y); break;
    case 5: select_body<5>(st, wi.y); break;
    case 6: select_body<6>(st, wi.y); break;
    case 7: select_body<7>(st, wi.y); break;
    default: select_body<8>(st, wi.y); break;
  }
}

hipError_t launch_init_eval_wide(const DevState &st, hipStream_t s) {
  with_wide_m(st.m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    if (vary_tasked(st))
      hipLaunchKernelGGL((k_teval<M, 1>), dim3(2 * st.nblk), dim3(kBlock), 0, s, st);
    else
      with_lanes(st, [&](auto lc) {
        constexpr int LPO = decltype(lc)::value;
        hipLaunchKernelGGL((k_eval<M, 1, LPO>), dim3(vary_blocks_of(st.n, LPO)), dim3(kBlock), 0, s, st);
      });
  });
  return hipGetLastError();
}

hipError_t launch_phase_wide(const DevState &st, int phase, hipStream_t s) {
  with_wide_m(st.m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    if (phase == 0) {
      if (vary_tasked(st))
        hipLaunchKernelGGL((k_tvary<M, 1>), dim3(vary_grid(st)), dim3(kBlock), 0, s, st);
      else
        with_lanes(st, [&](auto lc) {
          constexpr int LPO = decltype(lc)::value;
          hipLaunchKernelGGL((k_vary<M, 1, LPO>), dim3(vary_grid(st)), dim3(kBlock), 0, s, st);
        });
    } else if (phase == 1) {
      hipLaunchKernelGGL((k_op1<M>), dim3(st.nblk), dim3(kBlock), 0, s, st);
    } else {
      hipLaunchKernelGGL((k_select<M>), dim3(st.sel_blocks0 + st.sel_blocks1), dim3(kBlock), 0, s,
                         st);
    }
  });
  return hipGetLastError();
}

hipError_t launch_batch_phase_wide(const DevState *states, const int2 *work, int nwork, int phase,
                                   bool tasked, hipStream_t s) {
  if (phase == 0 && tasked)
    hipLaunchKernelGGL(k_tvary_batch_w, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 0)
    hipLaunchKernelGGL(k_vary_batch_w, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else if (phase == 1)
    hipLaunchKernelGGL(k_op1_batch_w, dim3(nwork), dim3(kBlock), 0, s, states, work);
  else
    hipLaunchKernelGGL(k_select_batch_w, dim3(nwork), dim3(kBlock), 0, s, states, work);
  return hipGetLastError();
}

hipError_t launch_front_flags_wide(const DevState &st, int pop, uint8_t *keep, hipStream_t s) {
  with_wide_m(st.m, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    const int chunk = front_chunk(st.n);
    hipLaunchKernelGGL((k_front_init<M>), dim3(st.nblk), dim3(kBlock), 0, s, st, pop, keep);
    hipLaunchKernelGGL((k_front<M>), dim3(st.nblk, (st.n + chunk - 1) / chunk), dim3(kBlock), 0, s, st,
                       pop, keep, chunk);
  });
  return hipGetLastError();
}

}  // namespace gmpea
