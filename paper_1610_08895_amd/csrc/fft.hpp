// LDS-resident Stockham FFT engine for power-of-two lengths 32 <= K <= 4096.
//
// A workgroup transforms W independent sequences of length K held in LDS.  The first
// pass reads its inputs straight from a load functor (global memory) and the last pass
// writes straight to a store functor, so each element crosses HBM once each way.  Passes
// are radix-RB (8, or 16 when the panel has at least one radix-16 job per thread) except
// a leading one of radix 2^(log2 K mod log2 RB) when log2 K is not a multiple of log2 RB.
//
// Pass with radix R after stride NS (the product of the radices already applied): job j
// of a sequence reads a[r] = X[j + r K/R], multiplies a[r] by w^{r k}, w = exp(s 2 pi i /
// (NS R)), k = j mod NS, applies an R-point DFT and writes Y[(j - k) R + k + r NS] = a[r].
// After the last pass (NS R = K) the output is the DFT in natural order at index
// j + r K/R.  s = -1 is the forward transform exp(-2 pi i k q / K); s = +1 the
// unnormalised inverse.
//
// LDS layout: WFAST = true stores sequence w of element e at e*W + w and gives
// consecutive threads consecutive w (columns of a row-major grid: coalesced W-wide global
// segments, conflict-free LDS); WFAST = false stores at w*K + e and gives consecutive
// threads consecutive e (rows).
#pragma once

#include "common.hpp"

namespace ri {

__host__ __device__ constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 v) {  // v * (DIR i)
  return DIR < 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2* a) {
  const float2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft8(float2* a) {
  constexpr float H = 0.70710678118654752440f;
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // o_k *= exp(DIR 2 pi i k / 8)
  if (DIR < 0) {
    o1 = make_float2(H * (o1.x + o1.y), H * (o1.y - o1.x));
    o3 = make_float2(H * (o3.y - o3.x), -H * (o3.x + o3.y));
  } else {
    o1 = make_float2(H * (o1.x - o1.y), H * (o1.x + o1.y));
    o3 = make_float2(-H * (o3.x + o3.y), H * (o3.x - o3.y));
  }
  o2 = mul_i<DIR>(o2);
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

// 16-point DFT as 4 x 4: index n = 4 n1 + n2, k = k1 + 4 k2; 4-point DFTs over n1, the
// twiddles exp(DIR 2 pi i n2 k1 / 16), 4-point DFTs over n2, then the transpose.
template <int DIR>
__device__ __forceinline__ void dft16(float2* a) {
  constexpr float C1 = 0.92387953251128675613f;  // cos(pi / 8)
  constexpr float S1 = 0.38268343236508977173f;  // sin(pi / 8)
  constexpr float H = 0.70710678118654752440f;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<DIR>(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  // slot 4 k1 + n2 now holds the k1-th output of column n2; twiddle by w^(n2 k1)
  auto tw = [](float2 v, float c, float sn) {  // v * (c + DIR i sn)
    return DIR < 0 ? make_float2(v.x * c + v.y * sn, v.y * c - v.x * sn)
                   : make_float2(v.x * c - v.y * sn, v.y * c + v.x * sn);
  };
  a[5] = tw(a[5], C1, S1);     // w^1
  a[6] = tw(a[6], H, H);       // w^2
  a[7] = tw(a[7], S1, C1);     // w^3
  a[9] = tw(a[9], H, H);       // w^2
  a[10] = mul_i<DIR>(a[10]);   // w^4
  a[11] = tw(a[11], -H, H);    // w^6
  a[13] = tw(a[13], S1, C1);   // w^3
  a[14] = tw(a[14], -H, H);    // w^6
  a[15] = tw(a[15], -C1, -S1); // w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<DIR>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
  // slot 4 k1 + k2 holds output k1 + 4 k2
  float2 t[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = a[4 * (k & 3) + (k >> 2)];
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = t[k];
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) dft2<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<DIR>(a);
  else dft16<DIR>(a);
}

template <int K, int W, int NT, int DIR, bool WFAST>
struct FftPanel {
  static constexpr int LOGK = clog2(K);
  static constexpr int RB = W * (K / 16) >= NT ? 16 : 8;  // radix of the passes after the first
  static constexpr int LB = clog2(RB);
  static constexpr int R0 = LOGK % LB == 0 ? RB : (1 << (LOGK % LB));
  static constexpr int NPASS = LOGK % LB == 0 ? LOGK / LB : LOGK / LB + 1;
  static constexpr int LDS_ELEMS = K * W;
  static_assert(K >= 32 && K <= 4096 && (K & (K - 1)) == 0, "K");
  static_assert(NPASS >= 2, "at least two passes");

  __device__ static __forceinline__ int idx(int w, int e) { return WFAST ? e * W + w : w * K + e; }

  template <int R>
  __device__ static __forceinline__ void split(int g, int& w, int& j) {
    if (WFAST) {
      w = g % W;
      j = g / W;
    } else {
      j = g % (K / R);
      w = g / (K / R);
    }
  }

  template <int R, bool FIRST, bool LAST, class Load, class Store>
  __device__ static __forceinline__ void pass(float2* lds, const float2* tw, int ns, Load& load, Store& store) {
    constexpr int JOBS = W * (K / R);
    constexpr int PER = (JOBS + NT - 1) / NT;
    float2 a[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int g = tid + p * NT;
      if ((JOBS % NT == 0) || g < JOBS) {
        int w, j;
        split<R>(g, w, j);
#pragma unroll
        for (int r = 0; r < R; ++r) a[p][r] = FIRST ? load(w, j + r * (K / R)) : lds[idx(w, j + r * (K / R))];
        if (!FIRST) {
          const int k = j & (ns - 1);
          const int step = k * (K / (ns * R));
          if constexpr (R == 16) {
            // w^r from the loaded w, w^2, w^4, w^8 (at most three roundings each), which
            // replaces eleven of the fifteen LDS reads of the table
            float2 w[16];
            w[1] = tw[step];
            w[2] = tw[2 * step];
            w[4] = tw[4 * step];
            w[8] = tw[8 * step];
            if (DIR > 0) {
              w[1].y = -w[1].y;
              w[2].y = -w[2].y;
              w[4].y = -w[4].y;
              w[8].y = -w[8].y;
            }
            w[3] = cmul(w[1], w[2]);
            w[5] = cmul(w[1], w[4]);
            w[6] = cmul(w[2], w[4]);
            w[7] = cmul(w[3], w[4]);
#pragma unroll
            for (int r = 1; r < 8; ++r) w[8 + r] = cmul(w[r], w[8]);
#pragma unroll
            for (int r = 1; r < R; ++r) a[p][r] = cmul(a[p][r], w[r]);
          } else if constexpr (R == 8) {  // likewise from w, w^2, w^4
            float2 w[8];
            w[1] = tw[step];
            w[2] = tw[2 * step];
            w[4] = tw[4 * step];
            if (DIR > 0) {
              w[1].y = -w[1].y;
              w[2].y = -w[2].y;
              w[4].y = -w[4].y;
            }
            w[3] = cmul(w[1], w[2]);
            w[5] = cmul(w[1], w[4]);
            w[6] = cmul(w[2], w[4]);
            w[7] = cmul(w[3], w[4]);
#pragma unroll
            for (int r = 1; r < R; ++r) a[p][r] = cmul(a[p][r], w[r]);
          } else {
#pragma unroll
            for (int r = 1; r < R; ++r) {
              float2 t = tw[r * step];
              if (DIR > 0) t.y = -t.y;
              a[p][r] = cmul(a[p][r], t);
            }
          }
        }
        dft<R, DIR>(a[p]);
      }
    }
    if (!FIRST) __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int g = tid + p * NT;
      if ((JOBS % NT == 0) || g < JOBS) {
        int w, j;
        split<R>(g, w, j);
        if (LAST) {
#pragma unroll
          for (int r = 0; r < R; ++r) store(w, j + r * (K / R), a[p][r]);
        } else {
          const int k = j & (ns - 1);
          const int base = (j - k) * R + k;
#pragma unroll
          for (int r = 0; r < R; ++r) lds[idx(w, base + r * ns)] = a[p][r];
        }
      }
    }
    if (!LAST) __syncthreads();
  }

  // tw: K forward twiddles exp(-2 pi i e / K) in global memory.  With TWL they are first
  // copied to twl (K entries of LDS) and read from there.
  template <bool TWL, class Load, class Store>
  __device__ static void run(float2* lds, const float2* __restrict__ tw, float2* twl, Load& load, Store& store) {
    if constexpr (TWL) {
      for (int e = threadIdx.x; e < K; e += NT) twl[e] = tw[e];
      passes(lds, twl, load, store);  // the first pass's barrier orders these writes before any read
    } else {
      passes(lds, tw, load, store);
    }
  }

  template <class Load, class Store>
  __device__ static __forceinline__ void passes(float2* lds, const float2* tw, Load& load, Store& store) {
    pass<R0, true, false>(lds, tw, 1, load, store);
    int ns = R0;
    if constexpr (NPASS >= 4) {
#pragma unroll 1
      for (int p = 1; p < NPASS - 1; ++p) {
        pass<RB, false, false>(lds, tw, ns, load, store);
        ns *= RB;
      }
    } else if constexpr (NPASS == 3) {
      pass<RB, false, false>(lds, tw, ns, load, store);
      ns *= RB;
    }
    pass<RB, false, true>(lds, tw, ns, load, store);
  }
};

}  // namespace ri
