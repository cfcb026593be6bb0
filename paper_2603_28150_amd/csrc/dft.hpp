// Small in-register DFTs (sizes 1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 27, 32)
// used by the 2D FFT kernels.
// DIR = -1: forward, exp(-2 pi i n k / R); DIR = +1: inverse (unnormalised).
#pragma once

#include <hip/hip_runtime.h>

namespace pat {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by exp(DIR * i pi / 2): -i (forward) or +i (inverse)
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// exp(DIR * 2 pi i e / 32) for 0 <= e < 16, from exact constants.
template <int DIR>
__device__ __forceinline__ float2 w32(int e) {
  const float cs[16] = {1.f,
                        0.98078528040323044913f, 0.92387953251128675613f, 0.83146961230254523708f,
                        0.70710678118654752440f, 0.55557023301960222474f, 0.38268343236508977173f,
                        0.19509032201612826785f, 0.f,
                        -0.19509032201612826785f, -0.38268343236508977173f, -0.55557023301960222474f,
                        -0.70710678118654752440f, -0.83146961230254523708f, -0.92387953251128675613f,
                        -0.98078528040323044913f};
  const float sn[16] = {0.f,
                        0.19509032201612826785f, 0.38268343236508977173f, 0.55557023301960222474f,
                        0.70710678118654752440f, 0.83146961230254523708f, 0.92387953251128675613f,
                        0.98078528040323044913f, 1.f,
                        0.98078528040323044913f, 0.92387953251128675613f, 0.83146961230254523708f,
                        0.70710678118654752440f, 0.55557023301960222474f, 0.38268343236508977173f,
                        0.19509032201612826785f};
  return make_float2(cs[e & 15], DIR < 0 ? -sn[e & 15] : sn[e & 15]);
}

// exp(DIR * 2 pi i e / 16) for 0 <= e < 16, from exact constants.
template <int DIR>
__device__ __forceinline__ float2 w16(int e) {
  constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
  constexpr float r2 = 0.70710678118654752440f;  // cos(pi/4)
  const float cs[16] = {1.f, c1, r2, s1, 0.f, -s1, -r2, -c1, -1.f, -c1, -r2, -s1, 0.f, s1, r2, c1};
  const float sn[16] = {0.f, s1, r2, c1, 1.f, c1, r2, s1, 0.f, -s1, -r2, -c1, -1.f, -c1, -r2, -s1};
  return make_float2(cs[e & 15], DIR < 0 ? -sn[e & 15] : sn[e & 15]);
}

// exp(DIR * 2 pi i e / 432), e >= 0, from cos(2 pi j / 432), j = 0..108 (a
// quarter period; 432 = 16 * 27 is a multiple of every small DFT size here)
__device__ __forceinline__ float cos432(int e) {
  const float c[109] = {
      1.f, 0.9998942319271075f, 0.9995769500822006f, 0.9990482215818578f, 0.9983081582712682f,
      0.9973569167005722f, 0.9961946980917455f, 0.9948217482960331f, 0.993238357741943f, 0.9914448613738104f,
      0.9894416385809445f, 0.987229113117374f, 0.984807753012208f, 0.9821780704706307f, 0.9793406217655515f,
      0.9762960071199334f, 0.9730448705798238f, 0.969587899878116f, 0.9659258262890683f, 0.9620594244736133f,
      0.9579895123154889f, 0.9537169507482269f, 0.9492426435730339f, 0.9445675372676048f, 0.9396926207859084f,
      0.9346189253489884f, 0.9293475242268224f, 0.9238795325112867f, 0.918216106880274f, 0.9123584453530141f,
      0.9063077870366499f, 0.9000654118641211f, 0.8936326403234123f, 0.8870108331782217f, 0.8802013911801111f,
      0.8732057547721958f, 0.8660254037844387f, 0.8586618571206132f, 0.8511166724369997f, 0.8433914458128857f,
      0.8354878114129365f, 0.8274074411415105f, 0.8191520442889918f, 0.8107233671702123f, 0.8021231927550438f,
      0.7933533402912352f, 0.7844156649195757f, 0.7753120572814658f, 0.766044443118978f, 0.756614782867493f,
      0.747025071240996f, 0.7372773368101241f, 0.7273736415730486f, 0.7173160805192894f, 0.7071067811865476f,
      0.696747903210655f, 0.6862416378687336f, 0.6755902076156604f, 0.6647958656139379f, 0.6538608952570697f,
      0.6427876096865395f, 0.6315783513024975f, 0.62023549126826f, 0.6087614290087207f, 0.5971585917027862f,
      0.5854294337699406f, 0.5735764363510462f, 0.561602106783493f, 0.549508978070806f, 0.5372996083468239f,
      0.5249765803345602f, 0.5125425007998652f, 0.5f, 0.4873517311272424f, 0.4746003697476404f,
      0.4617486132350341f, 0.4487991802004623f, 0.43575480991707943f, 0.42261826174069944f, 0.4093923145260925f,
      0.3960797660391569f, 0.38268343236508984f, 0.36920614731268464f, 0.3556507618148764f, 0.3420201433256686f,
      0.3283171752135611f, 0.31454475615161365f, 0.3007057995042733f, 0.2868032327110903f, 0.27283999666746106f,
      0.25881904510252074f, 0.24474334395432393f, 0.23061587074244025f, 0.21643961393810313f, 0.2022175723320379f,
      0.18795275440011178f, 0.17364817766693041f, 0.1593068680675226f, 0.14493185930724692f, 0.1305261922200515f,
      0.1160929141252303f, 0.10163507818280189f, 0.08715574274765836f, 0.07265797072261074f, 0.05814482891047568f,
      0.04361938736533601f, 0.02908471874311136f, 0.014543897651582776f, 0.f};
  e %= 432;
  return e <= 108 ? c[e] : e <= 216 ? -c[216 - e] : e <= 324 ? -c[e - 216] : c[432 - e];
}
template <int DIR>
__device__ __forceinline__ float2 w432(int e) {
  const float sn = cos432(e + 324);  // sin(t) = cos(t - 90 degrees)
  return make_float2(cos432(e), DIR < 0 ? -sn : sn);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// in place on v[0], v[s], v[2s], v[3s]
template <int DIR>
__device__ __forceinline__ void dft4(float2* v, int s) {
  float2 a0 = cadd(v[0], v[2 * s]), a1 = csub(v[0], v[2 * s]);
  float2 b0 = cadd(v[s], v[3 * s]), b1 = rot90<DIR>(csub(v[s], v[3 * s]));
  v[0] = cadd(a0, b0);
  v[2 * s] = csub(a0, b0);
  v[s] = cadd(a1, b1);
  v[3 * s] = csub(a1, b1);
}

// in place on a, b, c: X1 = a - (b+c)/2 + DIR i (sqrt(3)/2)(b-c), X2 its mirror
template <int DIR>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  constexpr float h = 0.8660254037844386f;  // sqrt(3)/2
  const float2 s = cadd(b, c), d = csub(b, c);
  const float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
  const float2 r = rot90<DIR>(cscale(d, h));
  a = cadd(a, s);
  b = cadd(m, r);
  c = csub(m, r);
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v);

// R = P * Q points (R dividing 432): input n = Q n1 + n2, output k = k1 + P k2;
// P-point DFTs over n1, twiddles exp(DIR 2 pi i n2 k1 / R), Q-point DFTs over n2
template <int P, int Q, int DIR>
__device__ __forceinline__ void dft_pq(float2* v) {
  constexpr int R = P * Q;
  static_assert(432 % R == 0, "twiddles come from the 432-point table");
  float2 y[R];
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    float2 t[P];
#pragma unroll
    for (int n1 = 0; n1 < P; ++n1) t[n1] = v[Q * n1 + n2];
    dft<P, DIR>(t);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1)
      y[n2 * P + k1] = (n2 * k1 == 0) ? t[k1] : cmul(t[k1], w432<DIR>(n2 * k1 * (432 / R)));
  }
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) {
    float2 t[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) t[n2] = y[n2 * P + k1];
    dft<Q, DIR>(t);
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = t[k2];
  }
}

// Full DFT of R points held in v[0..R-1]; natural order in and out.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(v[0], v[1], v[2]);
  } else if constexpr (R == 6 || R == 9 || R == 12 || R == 18 || R == 24 || R == 27) {
    dft_pq<R / 3, 3, DIR>(v);
  } else if constexpr (R == 4) {
    dft4<DIR>(v, 1);
  } else if constexpr (R == 8) {
    // radix 2 x 4: even/odd halves, then combine with exp(DIR 2 pi i k / 8)
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<DIR>(e, 1);
    dft4<DIR>(o, 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float2 t = cmul(o[k], w16<DIR>(2 * k));
      v[k] = cadd(e[k], t);
      v[k + 4] = csub(e[k], t);
    }
  } else if constexpr (R == 16) {
    // four-step 4 x 4: input n = n2 + 4 n1, output k = k1 + 4 k2
    float2 y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
      dft4<DIR>(t, 1);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2 * 4 + k1] = (n2 * k1 == 0) ? t[k1] : cmul(t[k1], w16<DIR>(n2 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {y[k1], y[4 + k1], y[8 + k1], y[12 + k1]};
      dft4<DIR>(t, 1);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  } else {
    static_assert(R == 32, "unsupported DFT size");
    // radix 2 x 16: even/odd halves, then combine with exp(DIR 2 pi i k / 32)
    float2 e[16], o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    dft<16, DIR>(e);
    dft<16, DIR>(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float2 t = k == 0 ? o[k] : cmul(o[k], w32<DIR>(k));
      v[k] = cadd(e[k], t);
      v[k + 16] = csub(e[k], t);
    }
  }
}

// Split of N = N1 * N2 used by the four-step kernels (N1 >= N2).
template <int N> struct Split;
template <> struct Split<16> { static constexpr int N1 = 4, N2 = 4; };
template <> struct Split<32> { static constexpr int N1 = 8, N2 = 4; };
template <> struct Split<64> { static constexpr int N1 = 8, N2 = 8; };
template <> struct Split<128> { static constexpr int N1 = 16, N2 = 8; };
template <> struct Split<256> { static constexpr int N1 = 16, N2 = 16; };
template <> struct Split<512> { static constexpr int N1 = 32, N2 = 16; };
template <> struct Split<1024> { static constexpr int N1 = 32, N2 = 32; };
template <> struct Split<48> { static constexpr int N1 = 8, N2 = 6; };
template <> struct Split<96> { static constexpr int N1 = 12, N2 = 8; };
template <> struct Split<192> { static constexpr int N1 = 16, N2 = 12; };
template <> struct Split<384> { static constexpr int N1 = 24, N2 = 16; };
template <> struct Split<768> { static constexpr int N1 = 32, N2 = 24; };
template <> struct Split<72> { static constexpr int N1 = 9, N2 = 8; };
template <> struct Split<108> { static constexpr int N1 = 12, N2 = 9; };
template <> struct Split<144> { static constexpr int N1 = 12, N2 = 12; };
template <> struct Split<216> { static constexpr int N1 = 18, N2 = 12; };
template <> struct Split<288> { static constexpr int N1 = 18, N2 = 16; };
template <> struct Split<432> { static constexpr int N1 = 24, N2 = 18; };
template <> struct Split<576> { static constexpr int N1 = 24, N2 = 24; };
template <> struct Split<864> { static constexpr int N1 = 32, N2 = 27; };

}  // namespace pat
