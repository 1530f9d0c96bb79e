// C ABI of libtcflow: argument checking, weight packing, buffer layouts and
// the launch sequence of the flow network and the consistency step.
#include <math.h>
#include <string.h>

#include <cmath>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/tcflow.h"
#include "tc_internal.h"

using namespace tc;

struct tc_net {
  tc_net_desc d;
  int precision;
  int bf16act;      // activations stored as bfloat16, convs on BF16 MFMA
  int fp8;          // convs on FP8 E4M3 MFMA (activations still stored as bfloat16)
  int f16feat;      // BF16/FP8 forms: pyramid features stored as float16 (the
                    // cost volume's inputs); the convs reading them convert
  int esz;          // bytes per stored activation element
  int ncv;          // (2r+1)^2
  int zcb;          // blocks of the cost-volume buffer (ncv + 2, rounded up to 8)
  ConvLayer pyr[8][2];
  ConvLayer dec[8][4];  // levels below d.finest have no estimator (unused)
  SepLayer ref[8];      // refinement layers 0 .. d.ref_layers - 1
  void* dmem;
};

namespace {

constexpr int kMaxN = 4096, kMaxHW = 16384;
constexpr int kHeadMaxIn = 128;  // 16 channel blocks of 8 (launch_head)
constexpr long kWino4Regions = 128;  // F(4x4, 3x3) from this many 16 x 32 regions per image
constexpr size_t kAlign = 256;

#define TC_TRY_HIP(x)                        \
  do {                                       \
    if ((x) != hipSuccess) return TC_ERR_HIP; \
  } while (0)

// ---- measurement probe (see tc_probe_enable)
struct Probe {
  int stage = -1;
  int count = 0;
  std::vector<hipEvent_t> ev;  // 2 per launch
};
Probe g_probe;

inline void probe_begin(int stage, hipStream_t s) {
  if (stage == g_probe.stage && 2 * g_probe.count < (int)g_probe.ev.size())
    (void)hipEventRecord(g_probe.ev[2 * g_probe.count], s);
}
inline void probe_end(int stage, hipStream_t s) {
  if (stage == g_probe.stage && 2 * g_probe.count < (int)g_probe.ev.size()) {
    (void)hipEventRecord(g_probe.ev[2 * g_probe.count + 1], s);
    ++g_probe.count;
  }
}

bool desc_ok(const tc_net_desc* d) {
  if (!d || d->levels < 1 || d->levels > 8) return false;
  for (int l = 0; l < d->levels; ++l)
    if (d->ch[l] <= 0 || d->ch[l] % 8 || d->ch[l] > 128) return false;
  for (int i = 0; i < 3; ++i)
    if (d->dec[i] <= 0 || d->dec[i] % 16 || d->dec[i] > 128) return false;
  // the estimator head (vector ALUs) takes at most kHeadMaxIn input channels
  if ((d->dec[1] + d->dec[2]) % 8 || d->dec[1] + d->dec[2] > kHeadMaxIn) return false;
  if (d->radius != 4) return false;
  if (!(d->leaky >= 0.f && d->leaky <= 1.f)) return false;
  if (d->finest < 1 || d->finest > d->levels) return false;
  if (d->ref_layers < 0 || d->ref_layers > 8) return false;
  int width = d->dec[1] + d->dec[2] + 2;
  for (int j = 0; j < d->ref_layers; ++j) {
    const bool last = j == d->ref_layers - 1;
    if (cdiv(width, 32) * 32 > kSepMaxC) return false;
    if (last ? d->ref_ch[j] != 2 : (d->ref_ch[j] <= 0 || d->ref_ch[j] % 8 || d->ref_ch[j] > 128))
      return false;
    if (d->ref_dil[j] < 1 || d->ref_dil[j] > 64) return false;
    width = d->ref_ch[j];
  }
  return true;
}

size_t conv_floats(int co, int ci) { return (size_t)co * ci * 9 + co; }

struct LevelDims {
  int hp, wp;             // padded input size
  int h[9], w[9];         // level sizes, index l = 1..L
};

LevelDims dims(const tc_net_desc& d, int h, int w) {
  LevelDims r;
  const int m = 1 << d.levels;
  r.hp = (h + m - 1) / m * m;
  r.wp = (w + m - 1) / m * m;
  for (int l = 1; l <= d.levels; ++l) {
    r.h[l] = r.hp >> l;
    r.w[l] = r.wp >> l;
  }
  return r;
}

bool shape_ok(int n, int h, int w) {
  return n > 0 && h > 0 && w > 0 && n <= kMaxN && h <= kMaxHW && w <= kMaxHW;
}

// ---- pyramid buffer layout: levels 1..L (blocked B = 8), then the staged
// frame (B = 4) and the scratch for each level's first conv.
struct PyrLayout {
  size_t off[9];
  size_t stage, tmp, partial, slots, total;
};

// amax slots (n images x kAmaxSub unsigned each): stage, then per level tmp
// and features
constexpr int kSub = 64 * 32;  // words per image (kAmaxWords of the kernels)
inline size_t pyr_slot(int n, int which) { return (size_t)which * n * kSub; }
inline int pyr_slot_stage() { return 0; }
inline int pyr_slot_tmp(int l) { return 1 + 2 * (l - 1); }
inline int pyr_slot_feat(int l) { return 2 + 2 * (l - 1); }

int layer_chunks(const ConvLayer& L) {
  return (L.bf16 || L.fp8) ? cdiv(L.cin_pad / 8, BF_CPC) : L.cin_pad / L.kc;
}

AmaxIn amax_plain(const unsigned* p) { return AmaxIn{p, p, 1 << 30}; }

size_t layer_partial_bytes(const ConvLayer& L, int out_h, int out_w, int n, int stride) {
  const ConvPlan p = plan_conv(out_h, out_w, n, layer_chunks(L), stride, L.np);
  return conv_partial_bytes(p, out_h, out_w, n, L.np);
}

PyrLayout pyr_layout(const tc_net* net, int n, int h, int w) {
  const tc_net_desc& d = net->d;
  PyrLayout p;
  LevelDims g = dims(d, h, w);
  size_t pos = 0, tmp = 0, part = 0;
  for (int l = 1; l <= d.levels; ++l) {
    const size_t bytes = (size_t)n * d.ch[l - 1] * g.h[l] * g.w[l] * net->esz;
    p.off[l] = pos;
    pos = align_up(pos + bytes, kAlign);
    if (bytes > tmp) tmp = bytes;
    for (int k = 0; k < 2; ++k) {
      const size_t pb = layer_partial_bytes(net->pyr[l - 1][k], g.h[l], g.w[l], n, k == 0 ? 2 : 1);
      if (pb > part) part = pb;
    }
  }
  p.stage = pos;
  // staged frame: float blocks of 4 or bfloat16 blocks of 8, 16 bytes per pixel
  pos = align_up(pos + (size_t)n * g.hp * g.wp * 16, kAlign);
  p.tmp = pos;
  pos = align_up(pos + tmp, kAlign);
  p.partial = pos;
  pos = align_up(pos + part, kAlign);
  p.slots = pos;
  pos = align_up(pos + (size_t)(1 + 2 * d.levels) * n * kSub * sizeof(unsigned), kAlign);
  p.total = pos;
  return p;
}

// ---- decoder scratch for a batch of nb images (n pairs -> nb = 2n)
struct DecLayout {
  size_t flow[2], U, Z, H1, H23, R[2], partial, slots, total;
};
// decoder amax slots (nb unsigned each): per level Z, H1, H2
inline int dec_slot(int l, int which) { return 3 * (l - 1) + which; }

DecLayout dec_layout(const tc_net* net, int nb, int h, int w) {
  DecLayout L;
  LevelDims g = dims(net->d, h, w);
  const int f = net->d.finest;
  const size_t px = (size_t)nb * g.h[f] * g.w[f];
  size_t pos = 0;
  auto take = [&](size_t bytes) {
    size_t o = pos;
    pos = align_up(pos + bytes, kAlign);
    return o;
  };
  L.flow[0] = take(px * 2 * sizeof(float));
  L.flow[1] = take(px * 2 * sizeof(float));
  L.U = take(px * 2 * sizeof(float));
  L.Z = take(px * net->zcb * 8 * net->esz);
  L.H1 = take(px * net->d.dec[0] * net->esz);
  // h2 | h3 (| the flow as one more block, the refinement's input)
  L.H23 = take(px * (net->d.dec[1] + net->d.dec[2] + (net->d.ref_layers ? 8 : 0)) * net->esz);
  int rw = 0;  // widest refinement activation (the last layer writes a flow)
  for (int j = 0; j + 1 < net->d.ref_layers; ++j) rw = std::max(rw, net->d.ref_ch[j]);
  L.R[0] = take(px * rw * net->esz);
  L.R[1] = take(px * rw * net->esz);
  size_t part = 0;
  for (int l = f; l <= net->d.levels; ++l)
    for (int k = 0; k < 4; ++k) {
      const size_t pb = layer_partial_bytes(net->dec[l - 1][k], g.h[l], g.w[l], nb, 1);
      if (pb > part) part = pb;
    }
  for (int l = f; l <= net->d.levels; ++l) {
    const size_t pb = cost_volume_partial_bytes(plan_cost_volume(g.h[l], g.w[l], net->d.ch[l - 1]),
                                                nb, g.h[l], g.w[l]);
    if (pb > part) part = pb;
  }
  L.partial = take(part);
  L.slots = take((size_t)3 * net->d.levels * nb * kSub * sizeof(unsigned));
  L.total = pos;
  return L;
}

// Pack W[cout][cin][3][3] (host, float) into [cin_pad/kc][9][kc][np] with the
// given map from packed input channel to source channel (-1 = zero).
void pack_conv(const float* W, const float* b, int cout, int cin, int kc, int cin_pad,
               const std::vector<int>& cmap, std::vector<float>& wout, std::vector<float>& bout,
               int& np) {
  np = (cout + 15) / 16 * 16;
  wout.assign((size_t)cin_pad * 9 * np, 0.f);
  bout.assign(np, 0.f);
  for (int g = 0; g < cin_pad; ++g) {
    const int c = cmap[g];
    if (c < 0) continue;
    const int chunk = g / kc, kk = g % kc;
    for (int tap = 0; tap < 9; ++tap)
      for (int o = 0; o < cout; ++o)
        wout[(((size_t)chunk * 9 + tap) * kc + kk) * np + o] = W[((size_t)o * cin + c) * 9 + tap];
  }
  for (int o = 0; o < cout; ++o) bout[o] = b[o];
}

uint16_t host_f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Pack W for conv3x3_bf16_mfma: per chunk of BF_CPC input blocks (8 channels
// each), the 9 * cpc (tap, block) pairs, block fastest, fill MFMA steps of 4
// lane groups: word [chunk][step][group][n] holds 8 bfloat16 k-values.
void pack_conv_bf16(const float* W, const float* b, int cout, int cin, int cin_pad,
                    const std::vector<int>& cmap, std::vector<uint16_t>& wout,
                    std::vector<float>& bout, int& np) {
  np = (cout + 15) / 16 * 16;
  const int nblk = cin_pad / 8, nch = cdiv(nblk, BF_CPC);
  wout.assign((size_t)nch * BF_STEPS * 4 * np * 8, 0);
  bout.assign(np, 0.f);
  for (int c = 0; c < nch; ++c) {
    const int cpc = std::min(BF_CPC, nblk - c * BF_CPC);
    for (int kb = 0; kb < 9 * cpc; ++kb) {
      const int tap = kb / cpc, cbi = kb % cpc, st = kb / 4, g = kb % 4;
      for (int o = 0; o < cout; ++o)
        for (int j = 0; j < 8; ++j) {
          const int src = cmap[(c * BF_CPC + cbi) * 8 + j];
          if (src < 0) continue;
          wout[((((size_t)c * BF_STEPS + st) * 4 + g) * np + o) * 8 + j] =
              host_f2bf(W[((size_t)o * cin + src) * 9 + tap]);
        }
    }
  }
  for (int o = 0; o < cout; ++o) bout[o] = b[o];
}

// float -> FP8 E4M3 as defined by the OCP 8-bit floating point specification
// ("E4M3FN": 1 sign, 4 exponent bits with bias 7, 3 mantissa bits, no
// infinities, largest finite 448, subnormals m/8 * 2^-6): round to nearest
// even, saturate to +-448, NaN -> 0x7f.
uint8_t host_f2e4m3(float f) {
  if (std::isnan(f)) return 0x7f;
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  const float a = std::fabs(f);
  if (a >= 448.f) return sign | 0x7e;
  int e2 = 0;
  std::frexp(a, &e2);  // a = m 2^e2, m in [0.5, 1)
  int E = e2 - 1;      // a = 1.xxx 2^E
  if (a == 0.f) return sign;
  if (E < -6) {        // subnormal: units of 2^-9
    const int q = (int)std::nearbyint(std::ldexp(a, 9));
    return sign | (uint8_t)q;  // q == 8 is the smallest normal, encoded 0x08
  }
  int q = (int)std::nearbyint(std::ldexp(a, 3 - E));  // in [8, 16]
  if (q == 16) {
    q = 8;
    ++E;
  }
  if (E + 7 > 15 || (E + 7 == 15 && q - 8 == 7)) return sign | 0x7e;
  return sign | (uint8_t)(((E + 7) << 3) | (q - 8));
}

// FP8 packing: the order of pack_conv_bf16, one byte per value, each output
// channel scaled by scale[o] = max|W[o]| / 448.
void pack_conv_fp8(const float* W, const float* b, int cout, int cin, int cin_pad,
                   const std::vector<int>& cmap, std::vector<uint8_t>& wout,
                   std::vector<float>& bout, std::vector<float>& scale, int& np) {
  np = (cout + 15) / 16 * 16;
  const int nblk = cin_pad / 8, nch = cdiv(nblk, BF_CPC);
  wout.assign((size_t)nch * BF_STEPS * 4 * np * 8, 0);
  bout.assign(np, 0.f);
  scale.assign(np, 1.f);
  for (int o = 0; o < cout; ++o) {
    float m = 0.f;
    for (int c = 0; c < cin * 9; ++c) m = std::max(m, std::fabs(W[(size_t)o * cin * 9 + c]));
    scale[o] = m > 0.f ? m / 448.f : 1.f;
  }
  for (int c = 0; c < nch; ++c) {
    const int cpc = std::min(BF_CPC, nblk - c * BF_CPC);
    for (int kb = 0; kb < 9 * cpc; ++kb) {
      const int tap = kb / cpc, cbi = kb % cpc, st = kb / 4, g = kb % 4;
      for (int o = 0; o < cout; ++o)
        for (int j = 0; j < 8; ++j) {
          const int src = cmap[(c * BF_CPC + cbi) * 8 + j];
          if (src < 0) continue;
          wout[((((size_t)c * BF_STEPS + st) * 4 + g) * np + o) * 8 + j] =
              host_f2e4m3(W[((size_t)o * cin + src) * 9 + tap] / scale[o]);
        }
    }
  }
  for (int o = 0; o < cout; ++o) bout[o] = b[o];
}

// FP8 packing for conv3x3_f8k128: per K step of 16 (tap, block) pairs
// (tap-major, k = tap * nblk + block, zero past the last pair), per lane
// group g and output channel n, the 8 channels of pairs 16 step + 4 g + j
// (j = 0..3), each output channel scaled by scale[o] (as pack_conv_fp8).
void pack_conv_f8k128(const float* W, int cout, int cin, int cin_pad, const std::vector<int>& cmap,
                      const std::vector<float>& scale, int np, std::vector<uint8_t>& wout,
                      int& nsteps) {
  const int nblk = cin_pad / 8, npairs = 9 * nblk;
  nsteps = f8k128_steps(cin_pad);
  wout.assign((size_t)nsteps * 4 * np * 32, 0);
  for (int s = 0; s < nsteps; ++s)
    for (int g = 0; g < 4; ++g)
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * s + 4 * g + j;
        if (k >= npairs) continue;
        const int tap = k / nblk, blk = k % nblk;
        for (int o = 0; o < cout; ++o)
          for (int c = 0; c < 8; ++c) {
            const int src = cmap[blk * 8 + c];
            if (src < 0) continue;
            wout[(((size_t)s * 4 + g) * np + o) * 32 + j * 8 + c] =
                host_f2e4m3(W[((size_t)o * cin + src) * 9 + tap] / scale[o]);
          }
      }
}

// Refinement layer packing.  Pointwise weights: per K chunk (16 channels for
// FP32, 32 for BF16), per 16-channel output block and lane l, the K/4 values
// W[16 nb + l % 16][K c + (K/4) (l / 16) + e] (float, or bfloat16), i.e. one
// MFMA B fragment per lane; zero for padded channels.  Input channels keep
// the order of the blob.
struct SepPacked {
  std::vector<char> pw;
  std::vector<float> rest;  // b [np], depthwise W [9][cin_pad], depthwise b [cin_pad],
                            // depthwise bfloat16 tap pairs [5][cin_pad] (bits)
};

void pack_sep(const SepLayer& L, const float* dw, const float* dwb, const float* pw,
              const float* pb, SepPacked& out) {
  const int K = L.bf16 ? 32 : 16, per = K / 4, nch = L.cin_pad / K, nbk = L.np / 16;
  const size_t nval = (size_t)nch * nbk * 64 * per;
  std::vector<float> wf(nval, 0.f);
  for (int c = 0; c < nch; ++c)
    for (int nb = 0; nb < nbk; ++nb)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < per; ++e) {
          const int o = nb * 16 + (l & 15), ch = c * K + per * (l >> 4) + e;
          if (o < L.cout && ch < L.cin)
            wf[(((size_t)c * nbk + nb) * 64 + l) * per + e] = pw[(size_t)o * L.cin + ch];
        }
  if (L.bf16) {
    out.pw.resize(nval * 2);
    for (size_t i = 0; i < nval; ++i) {
      const uint16_t v = host_f2bf(wf[i]);
      memcpy(out.pw.data() + 2 * i, &v, 2);
    }
  } else {
    out.pw.resize(nval * 4);
    memcpy(out.pw.data(), wf.data(), nval * 4);
  }
  out.rest.assign((size_t)L.np + 15 * L.cin_pad, 0.f);
  for (int o = 0; o < L.cout; ++o) out.rest[o] = pb[o];
  float* dwo = out.rest.data() + L.np;
  for (int c = 0; c < L.cin; ++c) {
    for (int tap = 0; tap < 9; ++tap) dwo[(size_t)tap * L.cin_pad + c] = dw[(size_t)c * 9 + tap];
    dwo[(size_t)9 * L.cin_pad + c] = dwb[c];
    for (int pr = 0; pr < 5; ++pr) {  // bfloat16 tap pairs for the BF16 form
      const uint32_t lo = host_f2bf(dw[(size_t)c * 9 + 2 * pr]);
      const uint32_t hi = 2 * pr + 1 < 9 ? host_f2bf(dw[(size_t)c * 9 + 2 * pr + 1]) : 0u;
      const uint32_t word = lo | (hi << 16);
      memcpy(dwo + (size_t)(10 + pr) * L.cin_pad + c, &word, 4);
    }
  }
}

View plain_view(const float* p, int cbt, int cb0 = 0) {
  View v;
  v.a = p;
  v.b = p;
  v.nsplit = 1 << 30;
  v.cbt = cbt;
  v.cb0 = cb0;
  v.tab = nullptr;
  return v;
}

int conv_layer(const ConvLayer& L, const View& in0, int nb0, const View& in1, int in_h, int in_w,
               float* out, int out_cbt, int out_cb0, int compact, const float* add, int out_h,
               int out_w, int relu, float slope, int n, int stride, int stage, float* partial,
               int act_bf16, const AmaxIn* ain, unsigned* aout, hipStream_t s, int in_f16 = 0,
               int out_f16 = 0) {
  ConvArgs a;
  a.in_f16 = in_f16;
  a.out_f16 = out_f16;
  a.in0 = in0;
  a.in1 = in1;
  a.nb0 = nb0;
  a.in_h = in_h;
  a.in_w = in_w;
  a.out = out;
  a.out_cbt = out_cbt;
  a.out_cb0 = out_cb0;
  a.compact = compact;
  a.add = add;
  a.out_h = out_h;
  a.out_w = out_w;
  a.w = L.w;
  a.b = L.b;
  a.nchunks = layer_chunks(L);
  a.nblk = L.cin_pad / 8;
  a.bf16act = (L.bf16 || L.fp8) ? 1 : 0;
  a.fp8 = L.fp8;
  a.wscale = L.ws;
  for (int i = 0; i < 3; ++i) a.ain[i] = ain ? ain[i] : AmaxIn{nullptr, nullptr, 0};
  a.aout = aout;
  a.cout = L.cout;
  a.np = L.np;
  a.lrelu = relu;
  a.slope = slope;
  a.n = n;
  a.partial = partial;
  hipError_t e;
  probe_begin(stage, s);
  if (L.cout == 2 && compact && stride == 1 && L.kc == 8 && !L.bf16 && !L.fp8) {
    // estimator head on vector ALUs (FP32 weights; BF16 activations are
    // multiplied as bfloat16 pairs)
    a.bf16act = act_bf16 ? 1 : 0;
    a.splits = 1;
    a.nchunks = L.cin_pad / 8;
    a.cps = a.nchunks;
    e = launch_head(a, s);
  } else {
    const ConvPlan p = plan_conv(out_h, out_w, n, a.nchunks, stride, L.np);
    a.splits = p.splits;
    a.cps = p.cps;
    // FP32 stride-1 layers with >= 32 tiles of 16 x 16 output pixels per
    // image (a per-image rule, so the choice never depends on the batch):
    // Winograd F(2x2, 3x3) on the matrix cores, without split K
    // F(4x4, 3x3) on layers with >= kWino4Regions regions of 16 x 32 output
    // pixels per image (also a per-image rule)
    if (L.wu4 && (long)cdiv(out_h, 16) * cdiv(out_w, 32) >= kWino4Regions &&
        wino_ok(a, stride, L.kc)) {
      a.splits = 1;
      a.cps = a.nchunks;
      e = launch_conv3x3_wino4(a, L.wu4, s);
    } else if (L.wu && (long)cdiv(out_h, 16) * cdiv(out_w, 16) >= 32 && wino_ok(a, stride, L.kc)) {
      a.splits = 1;
      a.cps = a.nchunks;
      e = launch_conv3x3_wino(a, L.wu, s);
    } else if (L.w8 && f8k128_ok(a, stride, p.mr, L.nsteps8)) {
      // FP8 on the K = 128 matrix instruction (layers without split K)
      e = launch_conv3x3_f8k128(a, L.w8, L.nsteps8, p.mr, s);
    } else
      e = launch_conv3x3(a, stride, L.kc, p.mr, s);
  }
  probe_end(stage, s);
  return e == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int run_pyramid(const tc_net* net, const float* frames, int n, int h, int w, char* pyr,
                hipStream_t s) {
  const tc_net_desc& d = net->d;
  const LevelDims g = dims(d, h, w);
  const PyrLayout p = pyr_layout(net, n, h, w);
  float* stage = reinterpret_cast<float*>(pyr + p.stage);
  float* tmp = reinterpret_cast<float*>(pyr + p.tmp);
  float* part = reinterpret_cast<float*>(pyr + p.partial);
  unsigned* slots = net->fp8 ? reinterpret_cast<unsigned*>(pyr + p.slots) : nullptr;
  auto slot = [&](int which) { return slots ? slots + pyr_slot(n, which) : nullptr; };
  if (slots) TC_TRY_HIP(launch_zero_u32(slots, (size_t)(1 + 2 * d.levels) * n * kSub, s));
  probe_begin(TC_STAGE_INPUT, s);
  TC_TRY_HIP(launch_stage(frames, n, h, w, stage, g.hp, g.wp, net->bf16act, nullptr, s));
  probe_end(TC_STAGE_INPUT, s);
  const float* in = stage;
  int in_cbt = 1, in_h = g.hp, in_w = g.wp;
  for (int l = 1; l <= d.levels; ++l) {
    const int C = d.ch[l - 1];
    float* feat = reinterpret_cast<float*>(pyr + p.off[l]);
    const ConvLayer& La = net->pyr[l - 1][0];
    const AmaxIn ain_a[3] = {amax_plain(slot(l == 1 ? pyr_slot_stage() : pyr_slot_feat(l - 1))),
                             {nullptr, nullptr, 0}, {nullptr, nullptr, 0}};
    const AmaxIn ain_b[3] = {amax_plain(slot(pyr_slot_tmp(l))), {nullptr, nullptr, 0},
                             {nullptr, nullptr, 0}};
    // level l >= 2 reads the float16 features of level l - 1
    const int fin = (l > 1 && net->f16feat) ? 1 : 0;
    int st = conv_layer(La, plain_view(in, in_cbt), La.cin_pad / ((La.bf16 || La.fp8) ? 8 : La.kc),
                        plain_view(in, in_cbt), in_h, in_w, tmp, C / 8, 0, 0, nullptr, g.h[l], g.w[l],
                        1, d.leaky, n, 2, TC_STAGE(l, TC_OP_PYR_A), part, net->bf16act, ain_a,
                        nullptr, s, fin, 0);
    if (st) return st;
    st = conv_layer(net->pyr[l - 1][1], plain_view(tmp, C / 8), C / 8, plain_view(tmp, C / 8),
                    g.h[l], g.w[l], feat, C / 8, 0, 0, nullptr, g.h[l], g.w[l], 1, d.leaky, n, 1,
                    TC_STAGE(l, TC_OP_PYR_B), part, net->bf16act, ain_b,
                    net->dec[l - 1][0].fp8 ? slot(pyr_slot_feat(l)) : nullptr, s, 0,
                    net->f16feat);
    if (st) return st;
    in = feat;
    in_cbt = C / 8;
    in_h = g.h[l];
    in_w = g.w[l];
  }
  return TC_OK;
}

// Per-image buffers of a batched decoder pass over separately stored pyramids:
// device tables (in the workspace) of level bases and output flows.
struct ListTables {
  const void* const* tab[9];  // per level: F1 bases of the nb images, then F2 bases
  float* const* out;          // nb output flows
};

// Decoder pass over nb = n (one direction) or 2n (both) images.
int run_decoder(const tc_net* net, const char* pyr1, const char* pyr2, int n, int h, int w,
                float* flow12, float* flow21, char* ws, hipStream_t s,
                const ListTables* lists = nullptr) {
  const tc_net_desc& d = net->d;
  const LevelDims g = dims(d, h, w);
  const PyrLayout p = pyr_layout(net, n, h, w);
  const int nb = flow21 ? 2 * n : n;
  const DecLayout D = dec_layout(net, nb, h, w);
  float* flows[2] = {reinterpret_cast<float*>(ws + D.flow[0]), reinterpret_cast<float*>(ws + D.flow[1])};
  float* U = reinterpret_cast<float*>(ws + D.U);
  float* Z = reinterpret_cast<float*>(ws + D.Z);
  float* H1 = reinterpret_cast<float*>(ws + D.H1);
  float* H23 = reinterpret_cast<float*>(ws + D.H23);
  float* part = reinterpret_cast<float*>(ws + D.partial);
  unsigned* dslots = net->fp8 ? reinterpret_cast<unsigned*>(ws + D.slots) : nullptr;
  auto dslot = [&](int l, int which) {
    return dslots ? dslots + (size_t)dec_slot(l, which) * nb * kSub : nullptr;
  };
  const unsigned* pslots1 =
      (net->fp8 && pyr1) ? reinterpret_cast<const unsigned*>(pyr1 + p.slots) : nullptr;
  const unsigned* pslots2 =
      (net->fp8 && pyr2) ? reinterpret_cast<const unsigned*>(pyr2 + p.slots) : nullptr;
  if (dslots) TC_TRY_HIP(launch_zero_u32(dslots, (size_t)3 * d.levels * nb * kSub, s));
  const AmaxIn none{nullptr, nullptr, 0};
  const int d0b = d.dec[0] / 8, d1b = d.dec[1] / 8, d23b = (d.dec[1] + d.dec[2]) / 8;
  const int hcb = d23b + (d.ref_layers ? 1 : 0);  // blocks per image of H23
  int cur = 0;
  const int fl = d.finest;
  for (int l = d.levels; l >= fl; --l) {
    const int C = d.ch[l - 1], hl = g.h[l], wl = g.w[l];
    const float* P1 = pyr1 ? reinterpret_cast<const float*>(pyr1 + p.off[l]) : nullptr;
    const float* P2 = pyr2 ? reinterpret_cast<const float*>(pyr2 + p.off[l]) : nullptr;
    View f1, f2;
    f1.a = P1; f1.b = P2; f1.nsplit = n; f1.cbt = C / 8; f1.cb0 = 0; f1.tab = nullptr;
    f2.a = P2; f2.b = P1; f2.nsplit = n; f2.cbt = C / 8; f2.cb0 = 0; f2.tab = nullptr;
    if (lists) {  // per-image pyramids: tables [F1 of 2n images | F2 of 2n images]
      f1.tab = lists->tab[l];
      f2.tab = lists->tab[l] + nb;
    }
    const float* Ul = nullptr;
    if (l < d.levels) {
      probe_begin(TC_STAGE(l, TC_OP_UP2), s);
      TC_TRY_HIP(launch_up2x2(flows[cur], nb, g.h[l + 1], g.w[l + 1], U, s));
      probe_end(TC_STAGE(l, TC_OP_UP2), s);
      Ul = U;
    }
    CvArgs cv;
    cv.f1 = f1;
    cv.f2 = f2;
    cv.U = Ul;
    cv.Z = Z;
    cv.zcb = net->zcb;
    cv.n = nb;
    cv.h = hl;
    cv.w = wl;
    cv.C = C;
    cv.radius = d.radius;
    cv.slope = d.leaky;
    const CvPlan cp = plan_cost_volume(hl, wl, C);
    cv.splits = cp.splits;
    cv.cps = cp.cps;
    cv.partial = part;
    cv.bf16act = net->bf16act;
    cv.f16feat = net->f16feat;
    cv.aout = net->dec[l - 1][0].fp8 ? dslot(l, 0) : nullptr;
    probe_begin(TC_STAGE(l, TC_OP_COST_VOLUME), s);
    TC_TRY_HIP(launch_warp_cost_volume(cv, s));
    probe_end(TC_STAGE(l, TC_OP_COST_VOLUME), s);
    const ConvLayer* L = net->dec[l - 1];
    // F1 of images [0, n) is pyr1's level l, of [n, 2n) pyr2's
    const AmaxIn fa{pslots1 ? pslots1 + pyr_slot(n, pyr_slot_feat(l)) : nullptr,
                    pslots2 ? pslots2 + pyr_slot(n, pyr_slot_feat(l)) : nullptr, n};
    const AmaxIn ain_c1[3] = {fa, amax_plain(dslot(l, 0)), none};
    const AmaxIn ain_c2[3] = {amax_plain(dslot(l, 1)), none, none};
    const AmaxIn ain_c3[3] = {amax_plain(dslot(l, 2)), none, none};
    // c1's K chunks: F1 (float16 features in the BF16/FP8 forms), then Z
    int st = conv_layer(L[0], f1, C / 8, plain_view(Z, net->zcb), hl, wl, H1, d0b, 0, 0, nullptr,
                        hl, wl, 1, d.leaky, nb, 1, TC_STAGE(l, TC_OP_C1), part, net->bf16act,
                        ain_c1, L[1].fp8 ? dslot(l, 1) : nullptr, s, net->f16feat ? 1 : 0, 0);
    if (st) return st;
    st = conv_layer(L[1], plain_view(H1, d0b), d0b, plain_view(H1, d0b), hl, wl, H23, hcb, 0, 0,
                    nullptr, hl, wl, 1, d.leaky, nb, 1, TC_STAGE(l, TC_OP_C2), part, net->bf16act,
                    ain_c2, L[2].fp8 ? dslot(l, 2) : nullptr, s);
    if (st) return st;
    st = conv_layer(L[2], plain_view(H23, hcb), d1b, plain_view(H23, hcb), hl, wl, H23, hcb,
                    d1b, 0, nullptr, hl, wl, 1, d.leaky, nb, 1, TC_STAGE(l, TC_OP_C3), part, net->bf16act,
                    ain_c3, nullptr, s);
    if (st) return st;
    const int nxt = cur ^ 1;
    st = conv_layer(L[3], plain_view(H23, hcb), d23b, plain_view(H23, hcb), hl, wl, flows[nxt],
                    0, 0, 1, Ul, hl, wl, 0, 0.f, nb, 1, TC_STAGE(l, TC_OP_HEAD), part, net->bf16act,
                    nullptr, nullptr, s);
    if (st) return st;
    cur = nxt;
  }
  if (d.ref_layers > 0) {
    // refinement on [h2 | h3 | flow_f] (H23 still holds the finest level's
    // h2 and h3, the flow goes into its last block); the last layer writes
    // flow_f + increment
    const int hl = g.h[fl], wl = g.w[fl];
    char* R[2] = {ws + D.R[0], ws + D.R[1]};
    probe_begin(TC_STAGE(fl, TC_OP_REFINE), s);
    TC_TRY_HIP(launch_flow_to_block(flows[cur], nb, hl * wl, H23, hcb, d23b, net->bf16act, s));
    for (int j = 0; j < d.ref_layers; ++j) {
      const bool last = j == d.ref_layers - 1;
      SepArgs a;
      a.in = j == 0 ? static_cast<const void*>(H23) : R[(j - 1) & 1];
      a.in_cbt = j == 0 ? hcb : d.ref_ch[j - 1] / 8;
      a.nblk = a.in_cbt;
      a.n = nb;
      a.h = hl;
      a.w = wl;
      a.slope = d.leaky;
      a.lrelu = last ? 0 : 1;
      a.out = last ? static_cast<void*>(flows[cur ^ 1]) : R[j & 1];
      a.out_cbt = last ? 0 : d.ref_ch[j] / 8;
      a.add = last ? flows[cur] : nullptr;
      TC_TRY_HIP(launch_sepconv(net->ref[j], a, s));
    }
    probe_end(TC_STAGE(fl, TC_OP_REFINE), s);
    cur ^= 1;
  }
  probe_begin(TC_STAGE_OUTPUT, s);
  TC_TRY_HIP(launch_final_flow(flows[cur], nb, g.h[fl], g.w[fl], 1 << fl, flow12, flow21, n, h, w,
                                lists ? lists->out : nullptr, s));
  probe_end(TC_STAGE_OUTPUT, s);
  return TC_OK;
}

bool aligned(const void* p) { return ((uintptr_t)p % kAlign) == 0; }

}  // namespace

extern "C" {

const char* tc_status_str(int st) {
  switch (st) {
    case TC_OK: return "ok";
    case TC_ERR_INVALID_ARG: return "invalid argument";
    case TC_ERR_SHAPE: return "inconsistent descriptor or weight count";
    case TC_ERR_WORKSPACE: return "workspace too small or misaligned";
    case TC_ERR_UNSUPPORTED: return "unsupported precision or size";
    case TC_ERR_HIP: return "HIP runtime or launch error";
    case TC_ERR_SCRATCH:
      return "input needs more than the no-allocation entry point's static scratch";
    default: return "unknown status";
  }
}

const char* tc_version(void) { return "tcflow 0.4 (gfx950; FP32, BF16 and FP8 E4M3 MFMA)"; }

void tc_fp8_e4m3_encode(const float* in, unsigned char* out, size_t n) {
  if (!in || !out) return;
  for (size_t i = 0; i < n; ++i) out[i] = host_f2e4m3(in[i]);
}

size_t tc_weight_floats(const tc_net_desc* d) {
  if (!desc_ok(d)) return 0;
  const int ncv = (2 * d->radius + 1) * (2 * d->radius + 1);
  size_t n = 0;
  for (int l = 1; l <= d->levels; ++l) {
    const int cin = l == 1 ? 3 : d->ch[l - 2];
    n += conv_floats(d->ch[l - 1], cin) + conv_floats(d->ch[l - 1], d->ch[l - 1]);
  }
  for (int l = d->finest; l <= d->levels; ++l) {
    n += conv_floats(d->dec[0], ncv + d->ch[l - 1] + 2) + conv_floats(d->dec[1], d->dec[0]) +
         conv_floats(d->dec[2], d->dec[1]) + conv_floats(2, d->dec[1] + d->dec[2]);
  }
  int width = d->dec[1] + d->dec[2] + 2;
  for (int j = 0; j < d->ref_layers; ++j) {
    n += (size_t)width * 9 + width + (size_t)d->ref_ch[j] * width + d->ref_ch[j];
    width = d->ref_ch[j];
  }
  return n;
}

int tc_net_create(const tc_net_desc* desc, const float* host_weights, size_t n_floats,
                  int precision, tc_net** out) {
  if (!desc || !host_weights || !out) return TC_ERR_INVALID_ARG;
  if (!desc_ok(desc)) return TC_ERR_SHAPE;
  const int base_prec = precision & ~TC_PREC_BF16_FEATURES;
  if ((base_prec != TC_FP32 && base_prec != TC_BF16 && base_prec != TC_FP8_E4M3) ||
      (base_prec == TC_FP32 && (precision & TC_PREC_BF16_FEATURES)))
    return TC_ERR_UNSUPPORTED;
  if (n_floats != tc_weight_floats(desc)) return TC_ERR_SHAPE;
  tc_net* net = new (std::nothrow) tc_net();
  if (!net) return TC_ERR_HIP;
  net->d = *desc;
  net->precision = precision;
  net->bf16act = base_prec == TC_BF16 || base_prec == TC_FP8_E4M3;
  net->fp8 = base_prec == TC_FP8_E4M3;
  net->f16feat = net->bf16act && !(precision & TC_PREC_BF16_FEATURES);
  net->esz = net->bf16act ? 2 : 4;
  net->ncv = (2 * desc->radius + 1) * (2 * desc->radius + 1);
  net->zcb = (net->ncv + 2 + 7) / 8;
  const int L = desc->levels;

  // host packing
  struct Packed {
    std::vector<char> w;
    std::vector<float> b;
    std::vector<float> sc;  // FP8 per-output-channel weight scales
    std::vector<float> wu;  // Winograd-transformed weights (FP32 stride-1 layers)
    std::vector<float> wu4;  // the same for F(4x4, 3x3)
    std::vector<uint8_t> w8;  // FP8 layers: the K = 128 MFMA packing
    int nsteps8 = 0;
  };
  std::vector<Packed> packed;
  std::vector<ConvLayer*> slots;
  const float* src = host_weights;
  // FP8 form: FP8 for the estimator convs of the two finest levels (most of
  // the FLOPs); the pyramid, whose features feed every cost volume, and the
  // coarse levels, whose errors are amplified by every upsampling on the way
  // to full resolution, stay BF16.
  auto add_layer = [&](ConvLayer& cl, int cout, int cin, int kc, int cin_pad,
                       const std::vector<int>& cmap, bool head, bool fp8_ok, bool stride1) {
    const float* W = src;
    const float* b = src + (size_t)cout * cin * 9;
    src += conv_floats(cout, cin);
    Packed pk;
    int np = 0;
    cl.fp8 = net->fp8 && !head && fp8_ok;
    cl.bf16 = net->bf16act && !cl.fp8 && !head;  // heads: FP32 packing for the vector-ALU head
    cl.ws = nullptr;
    if (cl.fp8) {
      std::vector<uint8_t> wq;
      pack_conv_fp8(W, b, cout, cin, cin_pad, cmap, wq, pk.b, pk.sc, np);
      pk.w.resize(wq.size());
      memcpy(pk.w.data(), wq.data(), pk.w.size());
      if (stride1) pack_conv_f8k128(W, cout, cin, cin_pad, cmap, pk.sc, np, pk.w8, pk.nsteps8);
    } else if (cl.bf16) {
      std::vector<uint16_t> wb;
      pack_conv_bf16(W, b, cout, cin, cin_pad, cmap, wb, pk.b, np);
      pk.w.resize(wb.size() * 2);
      memcpy(pk.w.data(), wb.data(), pk.w.size());
    } else {
      std::vector<float> wf;
      pack_conv(W, b, cout, cin, kc, cin_pad, cmap, wf, pk.b, np);
      pk.w.resize(wf.size() * 4);
      memcpy(pk.w.data(), wf.data(), pk.w.size());
      if (stride1 && !head && kc == 8 && cout % 32 == 0)
      {
        pack_conv_wino(W, cout, cin, cin_pad, cmap, pk.wu);
        pack_conv_wino4(W, cout, cin, cin_pad, cmap, pk.wu4);
      }
    }
    cl.cin = cin;
    cl.cout = cout;
    cl.cin_pad = cin_pad;
    cl.kc = kc;
    cl.np = np;
    packed.push_back(std::move(pk));
    slots.push_back(&cl);
  };
  auto identity = [](int cin, int pad) {
    std::vector<int> m(pad, -1);
    for (int c = 0; c < cin; ++c) m[c] = c;
    return m;
  };
  for (int l = 1; l <= L; ++l) {
    const int C = desc->ch[l - 1];
    const int cin = l == 1 ? 3 : desc->ch[l - 2];
    // the staged frame is one block of 4 (float) or 8 (bfloat16) channels
    const int kc = (l == 1 && !net->bf16act) ? 4 : 8;
    const int pad = l == 1 ? kc : cin;
    add_layer(net->pyr[l - 1][0], C, cin, kc, pad, identity(cin, pad), false, false, false);
    add_layer(net->pyr[l - 1][1], C, C, 8, C, identity(C, C), false, false, true);
  }
  const int d0 = desc->dec[0], d1 = desc->dec[1], d2 = desc->dec[2];
  for (int l = desc->finest; l <= L; ++l) {
    const int C = desc->ch[l - 1];
    // packed input order of c1: [F1 (C) | CV (ncv) | U (2) | zero pad];
    // source order of the blob: [CV (ncv) | F1 (C) | U (2)].
    const int pad = C + net->zcb * 8;
    std::vector<int> m(pad, -1);
    for (int g = 0; g < C; ++g) m[g] = net->ncv + g;
    for (int k = 0; k < net->ncv; ++k) m[C + k] = k;
    m[C + net->ncv] = net->ncv + C;
    m[C + net->ncv + 1] = net->ncv + C + 1;
    const bool f8 = l <= 2;
    add_layer(net->dec[l - 1][0], d0, net->ncv + C + 2, 8, pad, m, false, f8, true);
    add_layer(net->dec[l - 1][1], d1, d0, 8, d0, identity(d0, d0), false, f8, true);
    add_layer(net->dec[l - 1][2], d2, d1, 8, d1, identity(d1, d1), false, f8, true);
    add_layer(net->dec[l - 1][3], 2, d1 + d2, 8, d1 + d2, identity(d1 + d2, d1 + d2), true, false,
              true);
  }

  // refinement: per layer the pointwise weights packed as the sepconv kernel
  // reads them, then [b (np) | depthwise W (9 x cin_pad) | depthwise b]
  std::vector<SepPacked> sep(desc->ref_layers);
  {
    int cin = d1 + d2 + 2;  // [h2 | h3 | flow], the order of the blob
    for (int j = 0; j < desc->ref_layers; ++j) {
      SepLayer& sl = net->ref[j];
      const int cout = desc->ref_ch[j];
      sl.bf16 = net->bf16act;
      const int K = sl.bf16 ? 32 : 16;
      sl.cin = cin;
      sl.cin_pad = cdiv(cin, K) * K;
      sl.cout = cout;
      sl.np = cdiv(cout, 16) * 16;
      sl.dil = desc->ref_dil[j];
      const float* dw = src;
      const float* dwb = src + (size_t)cin * 9;
      const float* pw = dwb + cin;
      const float* pb = pw + (size_t)cout * cin;
      src = pb + cout;
      pack_sep(sl, dw, dwb, pw, pb, sep[j]);
      cin = cout;
    }
  }

  // one device allocation for every layer
  size_t total = 0;
  std::vector<size_t> offs;
  for (auto& pk : packed) {
    offs.push_back(total);
    total = align_up(total + pk.w.size(), kAlign);
    offs.push_back(total);
    total = align_up(total + (pk.b.size() + pk.sc.size()) * sizeof(float), kAlign);
    offs.push_back(total);
    total = align_up(total + pk.wu.size() * sizeof(float), kAlign);
    offs.push_back(total);
    total = align_up(total + pk.wu4.size() * sizeof(float), kAlign);
    offs.push_back(total);
    total = align_up(total + pk.w8.size(), kAlign);
  }
  for (auto& sp : sep) {
    offs.push_back(total);
    total = align_up(total + sp.pw.size(), kAlign);
    offs.push_back(total);
    total = align_up(total + sp.rest.size() * sizeof(float), kAlign);
  }
  if (hipMalloc(&net->dmem, total) != hipSuccess) {
    delete net;
    return TC_ERR_HIP;
  }
  std::vector<char> host(total, 0);
  for (size_t i = 0; i < packed.size(); ++i) {
    const size_t* o = &offs[5 * i];  // w, b (+ FP8 scales), wu, wu4, w8
    memcpy(host.data() + o[0], packed[i].w.data(), packed[i].w.size());
    memcpy(host.data() + o[1], packed[i].b.data(), packed[i].b.size() * sizeof(float));
    if (!packed[i].sc.empty())
      memcpy(host.data() + o[1] + packed[i].b.size() * sizeof(float), packed[i].sc.data(),
             packed[i].sc.size() * sizeof(float));
    if (!packed[i].wu.empty())
      memcpy(host.data() + o[2], packed[i].wu.data(), packed[i].wu.size() * sizeof(float));
    if (!packed[i].wu4.empty())
      memcpy(host.data() + o[3], packed[i].wu4.data(), packed[i].wu4.size() * sizeof(float));
    if (!packed[i].w8.empty()) memcpy(host.data() + o[4], packed[i].w8.data(), packed[i].w8.size());
    char* base = static_cast<char*>(net->dmem);
    slots[i]->w = reinterpret_cast<float*>(base + o[0]);
    slots[i]->b = reinterpret_cast<float*>(base + o[1]);
    if (slots[i]->fp8) slots[i]->ws = slots[i]->b + packed[i].b.size();
    slots[i]->wu = packed[i].wu.empty() ? nullptr : reinterpret_cast<float*>(base + o[2]);
    slots[i]->wu4 = packed[i].wu4.empty() ? nullptr : reinterpret_cast<float*>(base + o[3]);
    slots[i]->w8 = packed[i].w8.empty() ? nullptr : static_cast<void*>(base + o[4]);
    slots[i]->nsteps8 = packed[i].nsteps8;
  }
  for (size_t j = 0; j < sep.size(); ++j) {
    const size_t o0 = offs[5 * packed.size() + 2 * j], o1 = offs[5 * packed.size() + 2 * j + 1];
    memcpy(host.data() + o0, sep[j].pw.data(), sep[j].pw.size());
    memcpy(host.data() + o1, sep[j].rest.data(), sep[j].rest.size() * sizeof(float));
    SepLayer& sl = net->ref[j];
    char* base = static_cast<char*>(net->dmem);
    sl.pw = base + o0;
    sl.b = reinterpret_cast<float*>(base + o1);
    sl.dw = sl.b + sl.np;
    sl.dwb = sl.dw + (size_t)9 * sl.cin_pad;
    sl.dw2 = reinterpret_cast<const unsigned*>(sl.dwb + sl.cin_pad);
  }
  if (hipMemcpy(net->dmem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(net->dmem);
    delete net;
    return TC_ERR_HIP;
  }
  *out = net;
  return TC_OK;
}

void tc_net_destroy(tc_net* net) {
  if (!net) return;
  if (net->dmem) (void)hipFree(net->dmem);
  delete net;
}

size_t tc_pyramid_bytes(const tc_net* net, int n, int h, int w) {
  if (!net || !shape_ok(n, h, w)) return 0;
  return pyr_layout(net, n, h, w).total;
}

int tc_pyramid(const tc_net* net, const float* frames, int n, int h, int w, void* pyr,
               size_t pyr_bytes, hipStream_t stream) {
  if (!net || !frames || !pyr || !shape_ok(n, h, w)) return TC_ERR_INVALID_ARG;
  if (!aligned(pyr) || pyr_bytes < tc_pyramid_bytes(net, n, h, w)) return TC_ERR_WORKSPACE;
  return run_pyramid(net, frames, n, h, w, static_cast<char*>(pyr), (hipStream_t)stream);
}

size_t tc_decoder_workspace_bytes(const tc_net* net, int n, int h, int w) {
  if (!net || !shape_ok(n, h, w)) return 0;
  return dec_layout(net, 2 * n, h, w).total;
}

int tc_flow_from_pyramids(const tc_net* net, const void* pyr1, const void* pyr2, int n, int h,
                          int w, float* flow12, float* flow21, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  if (!net || !pyr1 || !pyr2 || !flow12 || !ws || !shape_ok(n, h, w)) return TC_ERR_INVALID_ARG;
  if (!aligned(ws) || !aligned(pyr1) || !aligned(pyr2)) return TC_ERR_WORKSPACE;
  if (ws_bytes < dec_layout(net, flow21 ? 2 * n : n, h, w).total) return TC_ERR_WORKSPACE;
  return run_decoder(net, static_cast<const char*>(pyr1), static_cast<const char*>(pyr2), n, h, w,
                     flow12, flow21, static_cast<char*>(ws), (hipStream_t)stream);
}

size_t tc_decoder_list_workspace_bytes(const tc_net* net, int n, int h, int w) {
  if (!net || !shape_ok(n, h, w) || n > kTabMax / 4) return 0;
  const size_t tables = (size_t)(net->d.levels * 4 * n + 2 * n) * sizeof(void*);
  return dec_layout(net, 2 * n, h, w).total + align_up(tables, kAlign);
}

int tc_flow_from_pyramid_list(const tc_net* net, const void* const* pyr_prev,
                              const void* const* pyr_cur, int n, int h, int w,
                              float* const* flow_fw, float* const* flow_bw, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (!net || !pyr_prev || !pyr_cur || !flow_fw || !flow_bw || !ws || !shape_ok(n, h, w))
    return TC_ERR_INVALID_ARG;
  if (n > kTabMax / 4) return TC_ERR_UNSUPPORTED;
  if (net->fp8) return TC_ERR_UNSUPPORTED;
  for (int i = 0; i < n; ++i)
    if (!pyr_prev[i] || !pyr_cur[i] || !flow_fw[i] || !flow_bw[i] || !aligned(pyr_prev[i]) ||
        !aligned(pyr_cur[i]))
      return TC_ERR_INVALID_ARG;
  if (!aligned(ws) || ws_bytes < tc_decoder_list_workspace_bytes(net, n, h, w))
    return TC_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const PyrLayout p = pyr_layout(net, 1, h, w);  // each listed pyramid holds one image
  const DecLayout D = dec_layout(net, 2 * n, h, w);
  char* base = static_cast<char*>(ws);
  const void** tabs = reinterpret_cast<const void**>(base + D.total);
  ListTables lt;
  // images [0, n) decode prev -> cur (forward), [n, 2n) cur -> prev (backward)
  for (int l = 1; l <= net->d.levels; ++l) {
    PtrTable t;
    for (int i = 0; i < n; ++i) {
      const char* a = static_cast<const char*>(pyr_prev[i]) + p.off[l];
      const char* b = static_cast<const char*>(pyr_cur[i]) + p.off[l];
      t.p[i] = a;          // F1, forward
      t.p[n + i] = b;      // F1, backward
      t.p[2 * n + i] = b;  // F2, forward
      t.p[3 * n + i] = a;  // F2, backward
    }
    const void** dst = tabs + (size_t)(l - 1) * 4 * n;
    TC_TRY_HIP(launch_write_table(t, 4 * n, dst, s));
    lt.tab[l] = dst;
  }
  {
    PtrTable t;
    for (int i = 0; i < n; ++i) {
      t.p[i] = flow_fw[i];
      t.p[n + i] = flow_bw[i];
    }
    const void** dst = tabs + (size_t)net->d.levels * 4 * n;
    TC_TRY_HIP(launch_write_table(t, 2 * n, dst, s));
    lt.out = reinterpret_cast<float* const*>(reinterpret_cast<void*>(dst));
  }
  return run_decoder(net, nullptr, nullptr, n, h, w, flow_fw[0], flow_bw[0], base, s, &lt);
}

size_t tc_flow_workspace_bytes(const tc_net* net, int n, int h, int w) {
  if (!net || !shape_ok(n, h, w)) return 0;
  return 2 * pyr_layout(net, n, h, w).total + dec_layout(net, 2 * n, h, w).total;
}

static int flow_common(const tc_net* net, const float* prev, const float* cur, int n, int h, int w,
                       float* f12, float* f21, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!net || !prev || !cur || !f12 || !ws || !shape_ok(n, h, w)) return TC_ERR_INVALID_ARG;
  if (!aligned(ws) || ws_bytes < tc_flow_workspace_bytes(net, n, h, w)) return TC_ERR_WORKSPACE;
  const size_t pb = pyr_layout(net, n, h, w).total;
  char* base = static_cast<char*>(ws);
  hipStream_t s = (hipStream_t)stream;
  int st = run_pyramid(net, prev, n, h, w, base, s);
  if (st) return st;
  st = run_pyramid(net, cur, n, h, w, base + pb, s);
  if (st) return st;
  return run_decoder(net, base, base + pb, n, h, w, f12, f21, base + 2 * pb, s);
}

int tc_flow_estimate(const tc_net* net, const float* prev, const float* cur, int n, int h, int w,
                     float* flow, void* ws, size_t ws_bytes, hipStream_t stream) {
  return flow_common(net, prev, cur, n, h, w, flow, nullptr, ws, ws_bytes, stream);
}

int tc_flow_estimate_pair(const tc_net* net, const float* prev, const float* cur, int n, int h,
                          int w, float* flow_fw, float* flow_bw, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  if (!flow_bw) return TC_ERR_INVALID_ARG;
  return flow_common(net, prev, cur, n, h, w, flow_fw, flow_bw, ws, ws_bytes, stream);
}

}  // extern "C"

// ---- the no-allocation entry point's scratch: one static array per device
// (every GPU the library runs on holds its own copy until the process ends).
// Host code never uses the array's name as an address: each device's address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address reaches kernels.
namespace {
static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for(hipStream_t s, void** out) {
  int dev = -1;
  if (s) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess) return TC_ERR_HIP;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return TC_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return TC_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return TC_ERR_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return TC_ERR_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return TC_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TC_OK;
}
}  // namespace

extern "C" {

int tc_flow_estimate_pair_noalloc(const tc_net* net, const float* prev, const float* cur, int n,
                                  int h, int w, float* flow_fw, float* flow_bw, hipStream_t stream) {
  if (!net || !prev || !cur || !flow_fw || !flow_bw || !shape_ok(n, h, w))
    return TC_ERR_INVALID_ARG;
  const size_t need = tc_flow_workspace_bytes(net, n, h, w);
  if (need > (size_t)TC_NOALLOC_SCRATCH_BYTES) return TC_ERR_SCRATCH;
  void* ptr = nullptr;
  const int st = scratch_for((hipStream_t)stream, &ptr);
  if (st) return st;
  return flow_common(net, prev, cur, n, h, w, flow_fw, flow_bw, ptr, need, stream);
}

size_t tc_flow_half_workspace_bytes(const tc_net* net, int n, int h, int w) {
  if (!net || !shape_ok(n, h, w)) return 0;
  const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
  const size_t fr = align_up((size_t)n * 3 * h2 * w2 * sizeof(float), kAlign);
  const size_t fl = align_up((size_t)n * 2 * h2 * w2 * sizeof(float), kAlign);
  return 2 * fr + 2 * fl + tc_flow_workspace_bytes(net, n, h2, w2);
}

int tc_flow_estimate_pair_half(const tc_net* net, const float* prev, const float* cur, int n,
                               int h, int w, float* flow_fw, float* flow_bw, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
  if (!net || !prev || !cur || !flow_fw || !flow_bw || !ws || !shape_ok(n, h, w))
    return TC_ERR_INVALID_ARG;
  if (!aligned(ws) || ws_bytes < tc_flow_half_workspace_bytes(net, n, h, w))
    return TC_ERR_WORKSPACE;
  const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
  const size_t fr = align_up((size_t)n * 3 * h2 * w2 * sizeof(float), kAlign);
  const size_t fl = align_up((size_t)n * 2 * h2 * w2 * sizeof(float), kAlign);
  char* base = static_cast<char*>(ws);
  float* a2 = reinterpret_cast<float*>(base);
  float* b2 = reinterpret_cast<float*>(base + fr);
  float* fw2 = reinterpret_cast<float*>(base + 2 * fr);
  float* bw2 = reinterpret_cast<float*>(base + 2 * fr + fl);
  char* rest = base + 2 * fr + 2 * fl;
  hipStream_t s = (hipStream_t)stream;
  TC_TRY_HIP(launch_half_frames(prev, 3 * n, h, w, a2, s));
  TC_TRY_HIP(launch_half_frames(cur, 3 * n, h, w, b2, s));
  const int st = flow_common(net, a2, b2, n, h2, w2, fw2, bw2, rest,
                             tc_flow_workspace_bytes(net, n, h2, w2), stream);
  if (st) return st;
  TC_TRY_HIP(launch_flow_up2_planes(fw2, n, h2, w2, h, w, flow_fw, s));
  TC_TRY_HIP(launch_flow_up2_planes(bw2, n, h2, w2, h, w, flow_bw, s));
  return TC_OK;
}

int tc_consistency_step(const float* stylized, const float* prev_out, const float* flow_fw,
                        const float* flow_bw, float alpha, int n, int h, int w, float* out,
                        unsigned char* mask_or_null, hipStream_t stream) {
  if (!stylized || !prev_out || !flow_fw || !flow_bw || !out) return TC_ERR_INVALID_ARG;
  if (!shape_ok(n, h, w)) return TC_ERR_INVALID_ARG;
  if (!(alpha >= 0.f && alpha <= 1.f)) return TC_ERR_INVALID_ARG;
  if (out == prev_out || out == flow_fw || out == flow_bw) return TC_ERR_INVALID_ARG;
  probe_begin(TC_STAGE_CONSISTENCY, (hipStream_t)stream);
  const hipError_t e = launch_consistency(stylized, prev_out, flow_fw, flow_bw, alpha, n, h, w,
                                          out, mask_or_null, (hipStream_t)stream);
  probe_end(TC_STAGE_CONSISTENCY, (hipStream_t)stream);
  return e == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int tc_flow_agreement(const float* flow_fw, const float* flow_bw, int n, int h, int w,
                      unsigned* counts, hipStream_t stream) {
  if (!flow_fw || !flow_bw || !counts || !shape_ok(n, h, w)) return TC_ERR_INVALID_ARG;
  return launch_agreement(flow_fw, flow_bw, n, h, w, counts, (hipStream_t)stream) == hipSuccess
             ? TC_OK
             : TC_ERR_HIP;
}

void tc_paper_default_params(tc_paper_params* p) {
  if (!p) return;
  p->k1 = 0.3f;
  p->k2 = 0.5f;
  p->a_ph = 6.5e3f;
  p->lambda = 2.0f;
  p->eta = 0.15f;
  p->kappa = 0.2f;
  p->iterations = 150;
}

int tc_paper_preset_params(int preset, tc_paper_params* p) {
  if (!p) return TC_ERR_INVALID_ARG;
  tc_paper_default_params(p);
  switch (preset) {
    case TC_PRESET_FINAL:
      return TC_OK;
    case TC_PRESET_OBJECTIVE:
      p->k1 = 0.3f;
      p->k2 = 0.3f;
      p->a_ph = 1.0e4f;
      p->lambda = 0.7f;
      return TC_OK;
    case TC_PRESET_FAST:
      p->iterations = 50;
      return TC_OK;
    default:
      return TC_ERR_INVALID_ARG;
  }
}

size_t tc_paper_workspace_bytes(int n, int h, int w) {
  if (!shape_ok(n, h, w)) return 0;
  return 16 * align_up((size_t)n * h * w * sizeof(float), kAlign);
}

int tc_consistency_paper(const float* I_prev, const float* I, const float* I_next,
                         const float* P_prev, const float* P, const float* P_next,
                         const float* O_prev, const float* flow_t_prev, const float* flow_t_next,
                         const tc_paper_params* prm, int n, int h, int w, float* out, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  if (!I_prev || !I || !I_next || !P_prev || !P || !P_next || !O_prev || !flow_t_prev ||
      !flow_t_next || !prm || !out || !ws || !shape_ok(n, h, w))
    return TC_ERR_INVALID_ARG;
  if (!(prm->k1 >= 0.f && prm->k2 >= 0.f && prm->k1 + prm->k2 <= 1.f && prm->a_ph >= 0.f &&
        prm->lambda >= 0.f && prm->eta >= 0.f && prm->kappa >= 0.f) ||
      prm->iterations < 0 || prm->iterations > 100000)
    return TC_ERR_INVALID_ARG;
  if (!aligned(ws) || ws_bytes < tc_paper_workspace_bytes(n, h, w)) return TC_ERR_WORKSPACE;
  const float* ins[] = {I_prev, I, I_next, P_prev, P, P_next, O_prev, flow_t_prev, flow_t_next};
  for (const float* q : ins)
    if (q == out) return TC_ERR_INVALID_ARG;
  const size_t pl = align_up((size_t)n * h * w * sizeof(float), kAlign);
  char* base = static_cast<char*>(ws);
  PaperArgs a;
  a.I_prev = I_prev; a.I = I; a.I_next = I_next;
  a.P_prev = P_prev; a.P = P; a.P_next = P_next;
  a.O_prev = O_prev; a.f_tp = flow_t_prev; a.f_tn = flow_t_next;
  a.k1 = prm->k1; a.k2 = prm->k2; a.a_ph = prm->a_ph; a.lambda = prm->lambda;
  a.eta = prm->eta; a.kappa = prm->kappa; a.iters = prm->iterations;
  a.n = n; a.h = h; a.w = w;
  a.R = reinterpret_cast<float*>(base);
  a.wc = reinterpret_cast<float*>(base + 3 * pl);
  a.O0 = reinterpret_cast<float*>(base + 4 * pl);
  a.O1 = reinterpret_cast<float*>(base + 7 * pl);
  a.O2 = reinterpret_cast<float*>(base + 10 * pl);
  a.O3 = reinterpret_cast<float*>(base + 13 * pl);
  hipStream_t s = (hipStream_t)stream;
  probe_begin(TC_STAGE_PAPER, s);
  const hipError_t e = launch_paper_step(a, out, 7, s);
  probe_end(TC_STAGE_PAPER, s);
  return e == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int tc_probe_enable(int stage, int max_launches) {
  if (max_launches <= 0 || max_launches > (1 << 20)) return TC_ERR_INVALID_ARG;
  tc_probe_disable();
  g_probe.ev.resize(2 * (size_t)max_launches);
  for (auto& e : g_probe.ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      tc_probe_disable();
      return TC_ERR_HIP;
    }
  g_probe.count = 0;
  g_probe.stage = stage;
  return TC_OK;
}

int tc_probe_read(int* launches, float* total_ms) {
  if (!launches || !total_ms) return TC_ERR_INVALID_ARG;
  float tot = 0.f;
  for (int i = 0; i < g_probe.count; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(g_probe.ev[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, g_probe.ev[2 * i], g_probe.ev[2 * i + 1]) != hipSuccess)
      return TC_ERR_HIP;
    tot += ms;
  }
  *launches = g_probe.count;
  *total_ms = tot;
  g_probe.count = 0;
  return TC_OK;
}

void tc_probe_disable(void) {
  for (auto& e : g_probe.ev)
    if (e) (void)hipEventDestroy(e);
  g_probe.ev.clear();
  g_probe.count = 0;
  g_probe.stage = -1;
}

}  // extern "C"
