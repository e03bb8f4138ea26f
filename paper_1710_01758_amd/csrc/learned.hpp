// Layout of the spectrum-correction network (internal, not part of the ABI).
#pragma once

#include "internal.hpp"

namespace pics {

constexpr int kNetGrid = 64;   // frequency grid of the network
constexpr int kNetFeat = 6;    // input feature planes
constexpr int kNetLayers = 6;  // 3x3 layers (a 1x1 layer follows)
constexpr float kNetFloor = 1e-3f;
constexpr int kWgRows = 4;  // image rows per workgroup of the weight gradient (partials per image: kNetGrid / kWgRows)

struct NetLayer {
  int cin, cinp, cout, dil;  // real / padded input channels, output channels, dilation
  long long woff;            // offset of W[cout][cin][3][3] in the flat parameters (bias follows)
  uint16_t* wf;              // bf16 [cout][9][cinp]
  uint16_t* wb;              // bf16 [cinp][9][cout]
};
struct NetLayout {
  NetLayer layer[kNetLayers];
  long long final_off;  // w[16], then bias
  long long count;      // total parameters
};

hipError_t launch_features(hipStream_t st, const Ws& w, int nslices, const float* energy, const float* kraw,
                           float* feat);
hipError_t launch_net_prep(hipStream_t st, const float* theta, const NetLayout& L);
hipError_t launch_net_input(hipStream_t st, const float* feat, const int* index, int batch, uint16_t* x0);
hipError_t launch_conv_fwd(hipStream_t st, int cinp, int cout, const uint16_t* x, const uint16_t* wf,
                           const float* bias, int dil, int batch, uint16_t* y);
hipError_t launch_conv_bwd_data(hipStream_t st, int cinp, int cout, const uint16_t* g, const uint16_t* wb,
                                const uint16_t* xact, int dil, int batch, uint16_t* gprev);
// part: batch * (kNetGrid / kWgRows) partial rows of cout * cin * 9 + cout
hipError_t launch_conv_bwd_w(hipStream_t st, int cinp, int cin, int cout, const uint16_t* x, const uint16_t* g,
                             int dil, int batch, float* part);
hipError_t launch_reduce_rows(hipStream_t st, const float* part, int rows, int count, float* grad);
hipError_t launch_net_head(hipStream_t st, const uint16_t* h6, const float* theta, int woff, const int* index,
                           int batch, const float* k, const float* G, const float* H, const float* Z,
                           const double* zsum, float* o, float* go, double* loss_part);
hipError_t launch_net_head_bwd(hipStream_t st, const uint16_t* h6, const float* theta, int woff, const float* go,
                               int batch, uint16_t* g6, float* part);
hipError_t launch_adam(hipStream_t st, float* theta, const float* g, float* m, float* v, int count, float lr, int t);
hipError_t launch_net_upsample(hipStream_t st, const Ws& w, const float* o, int slice0, int count,
                               long long max_pixels, float* corr);
hipError_t launch_probe_accum(const Simple& S, const Ws& w, const float2* fa, const float2* fz, float* G, float* H,
                              float* Z, float weight, int first);
hipError_t launch_plane_sums_indexed(hipStream_t st, const float* z, const int* index, int count, double* out);

}  // namespace pics
