// Wavefront-wide sums of doubles (wave64, gfx950) without LDS: DPP moves
// within 16-lane rows and v_permlane16/32_swap across rows.  Device code
// shared by the tall-skinny QR kernels and the batched CP-ALS-QR kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace cpqr {
namespace wave {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

__device__ __forceinline__ double rdlane(double x, int l) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), l));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ unsigned lo32(double x) {
  return unsigned(static_cast<unsigned long long>(__double_as_longlong(x)));
}
__device__ __forceinline__ unsigned hi32(double x) {
  return unsigned(static_cast<unsigned long long>(__double_as_longlong(x)) >> 32);
}
__device__ __forceinline__ double mkd(unsigned lo, unsigned hi) {
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// DPP lane moves within a row of 16 lanes: lanes of the enabled banks (groups
// of four lanes) take `src` from the lane CTRL names, the others keep `old`.
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_MIRROR = 0x140;      // lane i of a row takes lane 15 - i
constexpr int DPP_HALF_MIRROR = 0x141; // lane i of a half row takes lane 7 - i
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp(double old, double src) {
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(int(lo32(old)), int(lo32(src)), CTRL, 0xF, BANKS, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(int(hi32(old)), int(hi32(src)), CTRL, 0xF, BANKS, false));
  return mkd(lo, hi);
}

// Exchange across the halves of the wave (SPAN 32) or between neighbouring
// rows (SPAN 16).  The lanes with the SPAN bit clear get a from their partner
// lane (SPAN bit set) and keep their own a; the others get b from their
// partner and keep their own b; the two are summed.
template <int SPAN>
__device__ __forceinline__ double swap_sum(double a, double b) {
  if (SPAN == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
  }
}

// One level of the butterfly on lane bit B: the lanes with bit B clear keep
// (their a) + (partner's a), the others (their b) + (partner's b).  Bits 5
// and 4 use the permlane swaps, bits 3 and 2 the (half-)row mirrors, whose
// partner also differs in the lower bits; that is harmless because the lower
// bits are reduced afterwards.
template <int B>
__device__ __forceinline__ double bfly(double a, double b, int lane) {
  if (B == 5) return swap_sum<32>(a, b);
  if (B == 4) return swap_sum<16>(a, b);
  if (B == 3) return dpp<DPP_MIRROR, 0x3>(b, a) + dpp<DPP_MIRROR, 0xC>(a, b);
  if (B == 2) return dpp<DPP_HALF_MIRROR, 0x5>(b, a) + dpp<DPP_HALF_MIRROR, 0xA>(a, b);
  const bool hi = (lane >> B) & 1;
  const double send = hi ? a : b;
  return (hi ? b : a) + dpp<B == 1 ? DPP_XOR2 : DPP_XOR1, 0xF>(send, send);
}

// Sum over the 64 lanes of each x[i] (V a power of two <= 32): a
// reduce-scatter butterfly on lane bits 5, 4, ... splits the vector in half
// at each level, then the remaining lane bits are summed; sum i ends in the
// lanes whose bits 5 .. 6 - log2 V spell i, i.e. lanes (i << (6 - log2 V)) ..
// Returns the lane's sum, index lane >> (6 - log2 V).
template <int V, int LEV = 0>
__device__ __forceinline__ double wave_sum(double (&x)[V], int lane) {
  constexpr int L = ilog2(V);
  if constexpr (LEV < L) {
    constexpr int H = V >> (LEV + 1);
#pragma unroll
    for (int i = 0; i < H; ++i) x[i] = bfly<5 - LEV>(x[i], x[H + i], lane);
    return wave_sum<V, LEV + 1>(x, lane);
  } else if constexpr (LEV < 6) {
    x[0] = bfly<5 - LEV>(x[0], x[0], lane);
    return wave_sum<V, LEV + 1>(x, lane);
  } else {
    return x[0];
  }
}

// Sum over the 64 lanes, returned in every lane.
__device__ __forceinline__ double wave_allsum(double x, int lane) {
  x = bfly<5>(x, x, lane);
  x = bfly<4>(x, x, lane);
  x = bfly<3>(x, x, lane);
  x = bfly<2>(x, x, lane);
  x = bfly<1>(x, x, lane);
  return bfly<0>(x, x, lane);
}

}  // namespace wave
}  // namespace cpqr
