// Internal declarations shared by the HIP translation units of libtcflow.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace tc {

constexpr int kBlock = 256;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Activations are stored channel-blocked: element (img, c, y, x) of a buffer
// with `cbt` blocks of B channels per image lives at
//   base(img) + (((cb0 + c / B) * h + y) * w + x) * B + c % B
// so a block of B channels of one pixel is contiguous and neighbouring pixels
// are neighbouring in memory.  B = 8 everywhere except the staged RGB frame
// (B = 4).  A view may split its batch over two buffers: images [0, nsplit)
// come from `a`, the rest from `b` (index img - nsplit); or, when `tab` is
// set, image img lives in its own buffer tab[img] (a device-resident table).
struct View {
  const float* a;
  const float* b;
  int nsplit;
  int cbt;  // blocks per image in the underlying buffer
  int cb0;  // first block of the view
  const void* const* tab;
};

// Copies up to kTabMax pointers (carried in the kernel arguments) into a
// device-resident table.
constexpr int kTabMax = 64;
struct PtrTable {
  const void* p[kTabMax];
};
hipError_t launch_write_table(const PtrTable& t, int n, const void** dst, hipStream_t s);

// BF16 conv: channel blocks of 8 per K chunk and MFMA steps per full chunk.
constexpr int BF_CPC = 2;
constexpr int BF_STEPS = (9 * BF_CPC + 3) / 4;

// One 3x3 conv layer as the MFMA kernels consume it.  Weights are packed
// [cin_pad / kc][9 taps][kc][np] (tap = 3 * p + q), zero for padded input or
// output channels; np = cout rounded up to 16.  Bias has np entries.
struct ConvLayer {
  int cin, cout;   // real channel counts
  int cin_pad;     // multiple of kc
  int kc;          // input channels per K chunk (= block size of the input)
  int np;          // cout rounded up to 16
  float* w;        // device, packed (bfloat16 / FP8 bits for those layers)
  float* b;        // device, np floats
  int bf16;        // weights packed for conv3x3_bf16_mfma:
                   // [cdiv(cin_pad / 8, BF_CPC)][BF_STEPS][4][np][8] bfloat16
  int fp8;         // same order, FP8 E4M3 bytes, scaled per output channel by ws
  float* ws;       // device, np per-output-channel weight scales (FP8 layers)
  float* wu;       // device, Winograd-transformed weights (pack_conv_wino), or null
  float* wu4;      // device, F(4x4, 3x3) transformed weights (pack_conv_wino4), or null
  void* w8;        // device, FP8 weights for conv3x3_f8k128 (pack_conv_f8k128), or null
  int nsteps8;     // its K steps of 16 (tap, block) pairs
};

// Per-image absolute-maximum slots (float bits as unsigned) of an activation
// tensor: image img < nsplit uses a[img], else b[img - nsplit].  Producers
// fold their outputs into them; FP8 consumers derive their input scale.
struct AmaxIn {
  const unsigned* a;
  const unsigned* b;
  int nsplit;
};

struct ConvArgs {
  View in0, in1;  // K chunks [0, nb0) read in0, chunks [nb0, nchunks) read in1
  int nb0;
  int in_h, in_w;
  float* out;     // blocked output (B = 8) ...
  int out_cbt, out_cb0;
  int compact;    // ... or compact NHWC with `cout` channels when nonzero
  const float* add;  // compact NHWC (cout channels) added after the bias, or null
  int out_h, out_w;
  const float* w;
  const float* b;
  int nchunks, cout, np;
  int nblk;  // input channel blocks of 8 (bfloat16 path: a chunk holds 2 blocks)
  int lrelu;
  float slope;
  int n;  // images
  // split-K: grid z = n * splits; split s handles chunks [s * cps, (s+1) * cps)
  // and writes raw sums to partial[((s * n + img) * out_h + y) * out_w + x) * np + c];
  // a reduction pass then applies bias, LeakyReLU, `add` and the store.
  int splits, cps;
  float* partial;
  int bf16act;  // input and (blocked) output activations stored as bfloat16
  // ... except: bit v of in_f16 set = view v (in0, in1) stored as float16
  // (converted to bfloat16, or FP8, when staged); out_f16 = blocked output
  // stored as float16
  int in_f16, out_f16;
  int fp8;      // FP8 E4M3 MFMA: inputs scaled by max(ain) / 448, weights by wscale
  AmaxIn ain[3];
  const float* wscale;  // per output channel (np)
  unsigned* aout;       // per-image amax of the outputs, or null
};

// Launch plan of one conv: rows per wave (tile = 4 * mr rows x 16 columns)
// and the number of K splits.  Shared by workspace sizing and launching.
struct ConvPlan {
  int mr, splits, cps;
};
ConvPlan plan_conv(int out_h, int out_w, int n, int nchunks, int stride, int np);
size_t conv_partial_bytes(const ConvPlan& p, int out_h, int out_w, int n, int np);

hipError_t launch_conv3x3(const ConvArgs& a, int stride, int kc, int mr, hipStream_t s);
// FP32 stride-1 3x3 conv by Winograd F(2x2, 3x3) on the matrix cores
// (wino.hip): blocked outputs without `add`, cout a multiple of 8, np a
// multiple of 32, no split K.
bool wino_ok(const ConvArgs& a, int stride, int kc);
hipError_t launch_conv3x3_wino(const ConvArgs& a, const float* wu, hipStream_t s);
// The same layers by Winograd F(4x4, 3x3) (wino4.hip): 36 instead of 64
// products per 4x4 outputs and channel pair.
hipError_t launch_conv3x3_wino4(const ConvArgs& a, const float* wu4, hipStream_t s);
void pack_conv_wino4(const float* W, int cout, int cin, int cin_pad, const std::vector<int>& cmap,
                     std::vector<float>& out);
// FP8 E4M3 3x3 conv on the K = 128 FP8 MFMA (conv_f8.hip): stride 1, no
// split K, blocked outputs; the weights packed by pack_conv_f8k128 as
// [step][lane group (4)][n (np)][4 pairs x 8 channels] bytes, pair k = 16 step
// + 4 group + j taken tap-major (k = tap * nblk + block).
int f8k128_steps(int cin_pad);
bool f8k128_ok(const ConvArgs& a, int stride, int mr, int nsteps);
hipError_t launch_conv3x3_f8k128(const ConvArgs& a, const void* w8, int nsteps, int mr,
                                 hipStream_t s);
// 3x3 conv with two output channels (the estimator head) on vector ALUs,
// FP32 activations.
hipError_t launch_head(const ConvArgs& a, hipStream_t s);
// Host: the weights of launch_conv3x3_wino (G g G^T per channel pair).
void pack_conv_wino(const float* W, int cout, int cin, int cin_pad, const std::vector<int>& cmap,
                    std::vector<float>& out);


// NCHW float frames (n x 3 x h x w) -> one channel block per pixel, bottom /
// right edge replicated: float32 blocks of 4 (RGB, 0) or bfloat16 blocks of 8.
hipError_t launch_stage(const float* frames, int n, int h, int w, float* out, int hp, int wp,
                        int bf16act, unsigned* aout, hipStream_t s);

// Sets n unsigned words to zero (amax slots before a pass).
hipError_t launch_zero_u32(unsigned* p, size_t n, hipStream_t s);

// U = 2 * up2(flow), both compact NHWC with 2 channels: (n, h, w) -> (n, 2h, 2w).
hipError_t launch_up2x2(const float* flow, int n, int h, int w, float* U, hipStream_t s);

// Warp + cost volume: Z (blocked, B = 8, 11 blocks for radius 4) holds per
// pixel [lrelu(CV_k / C), k < 81 | U_x | U_y | 0 ...].  F1 and F2 are blocked
// pyramid levels with C / 8 blocks; U is compact NHWC (2 channels) or null
// for zero flow.
struct CvArgs {
  View f1, f2;
  const float* U;
  float* Z;
  int zcb;  // blocks per image of Z
  int n, h, w, C, radius;
  float slope;
  // channel split: grid z = n * splits, split s sums chunks [s * cps, (s+1) * cps)
  // into partial[((s * n + img) * 81 + k) * h * w + y * w + x]; a reduction
  // pass adds the splits in order and writes Z.
  int splits, cps;
  float* partial;
  int bf16act;  // features and Z stored as bfloat16
  int f16feat;  // with bf16act: features stored as float16, warped into float16
                // and correlated with float16 products and float32 sums (Z stays
                // bfloat16)
  unsigned* aout;  // per-image amax of the cost-volume outputs, or null
};
struct CvPlan {
  int splits, cps;
};
CvPlan plan_cost_volume(int h, int w, int C);
size_t cost_volume_partial_bytes(const CvPlan& p, int n, int h, int w);
hipError_t launch_warp_cost_volume(const CvArgs& a, hipStream_t s);

// Output: flow NCHW (n x 2 x H x W) = crop(s * upsample(flow_f, s)) with
// s = 2^finest (bilinear, half-pixel centres); flow_f NHWC (n x hf x wf x 2).
// Images [0, nsplit) go to out_a, the rest to out_b.
// Fast-preset resampling: 2x2 block means of `planes` h x w planes into
// ceil(h/2) x ceil(w/2) planes; flow planes (n x 2 x h2 x w2) upsampled to
// H x W with half-pixel centres and multiplied by 2.
hipError_t launch_half_frames(const float* in, int planes, int h, int w, float* out,
                              hipStream_t s);
hipError_t launch_flow_up2_planes(const float* in, int n, int h2, int w2, int H, int W, float* out,
                                  hipStream_t s);
hipError_t launch_final_flow(const float* flow_f, int n, int hf, int wf, int scale, float* out_a,
                             float* out_b, int nsplit, int H, int W, float* const* out_tab,
                             hipStream_t s);

// One depthwise separable layer of the refinement network: a depthwise 3x3
// conv with dilation `dil` (zero padding), bias and LeakyReLU, then a
// pointwise conv (bias, optional LeakyReLU).  The input channels are the
// first `nblk` blocks of the blocked buffer `in` (T = float, or bfloat16 with
// `bf16`); channels beyond them up to cin_pad have zero weights.  Output:
// blocked activations, or (cout = 2, `add` set) the flow add + result in
// NHWC float2.
constexpr int kSepMaxC = 256;          // padded input channels
constexpr int kSepPwFloats = 16384;    // pointwise weights held in LDS (64 KiB)
struct SepLayer {
  int cin, cin_pad, cout, np, dil;
  int bf16;         // BF16 operands (chunks of 32 channels), else FP32 (16)
  float* dw;        // device [9][cin_pad] depthwise weights (tap = 3 p + q), FP32
  float* dwb;       // device [cin_pad]
  const unsigned* dw2;  // device [5][cin_pad]: bfloat16 pairs (w[c][2p], w[c][2p+1]), w[c][9] = 0
  void* pw;         // device, packed [cin_pad / chunk][np / 16][64 lanes][chunk / 4]
  float* b;         // device [np]
};
struct SepArgs {
  const void* in;
  int in_cbt, nblk;
  int n, h, w;
  float slope;
  int lrelu;
  void* out;
  int out_cbt;
  const float* add;
};
hipError_t launch_sepconv(const SepLayer& L, const SepArgs& a, hipStream_t s);

// Writes the flow (NHWC float2) as channel block `cb` of a blocked buffer with
// `cbt` blocks per image (channels 0, 1 = the flow, 2..7 = 0), float or
// bfloat16.
hipError_t launch_flow_to_block(const float* flow, int n, int hw, void* out, int cbt, int cb,
                                int as_bf16, hipStream_t s);

// The paper's consistency step (Eq. 1-8).  Frames NCHW (n x 3 x h x w),
// flows n x 2 x h x w: f_tp = flow from t to t-1, f_tn = flow from t to t+1.
// Workspace planes: R (3), wc (1), O0..O3 (3 each).
struct PaperArgs {
  const float *I_prev, *I, *I_next, *P_prev, *P, *P_next, *O_prev, *f_tp, *f_tn;
  float k1, k2, a_ph, lambda, eta, kappa;
  int iters;
  int n, h, w;
  float *R, *wc, *O0, *O1, *O2, *O3;
};
hipError_t launch_paper_step(const PaperArgs& a, float* out, int block_iters, hipStream_t s);

// counts[i] = pixels of image i passing the forward-backward test of the
// consistency step (flows n x 2 x h x w).
hipError_t launch_agreement(const float* ffw, const float* fbw, int n, int h, int w,
                            unsigned* counts, hipStream_t s);

hipError_t launch_consistency(const float* P, const float* Oprev, const float* ffw,
                              const float* fbw, float alpha, int n, int h, int w, float* out,
                              unsigned char* mask, hipStream_t s);

// XCD-aware tile order.  Workgroup b of a grid (x fastest, then y, then z)
// runs on XCD b % 8 of the eight; each XCD is given a contiguous row-major
// range of the grid's tiles, so the halo that neighbouring tiles share is read
// into one L2.  Returns the tile (x, y, z) this workgroup computes (a
// bijection of the grid).
__device__ inline uint3 xcd_tile() {
  const unsigned gxy = gridDim.x * gridDim.y, total = gxy * gridDim.z;
  const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned q = total / 8, r = total % 8, xc = bid % 8;
  const unsigned wid = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + bid / 8;
  const unsigned z = wid / gxy, xy = wid - z * gxy, y = xy / gridDim.x;
  return make_uint3(xy - y * gridDim.x, y, z);
}

}  // namespace tc
