// Host check of which set-ups the single-pass kernel takes (no GPU needed):
// prints "<name> <0|1>" per case.
#include <cstdio>
#include <cstring>

#include "kernels_fused.h"

static lbm_params box(int nx, int ny, int nz, int precision, int zkind) {
  lbm_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = nx; p.ny = ny; p.nz = nz;
  p.precision = (lbm_precision)precision;
  for (int k = 0; k < 6; ++k) p.face[k] = LBM_FACE_PERIODIC;
  p.face[4] = p.face[5] = (lbm_face_kind)zkind;
  return p;
}

int main() {
  struct Case { const char* name; lbm_params p; };
  lbm_params outlet = box(512, 512, 384, LBM_FP32_DEV, LBM_FACE_WALL);
  outlet.face[5] = LBM_FACE_PRESSURE;
  lbm_params half_open = box(256, 256, 256, LBM_FP32_DEV, LBM_FACE_PRESSURE);
  half_open.face[5] = LBM_FACE_PERIODIC;
  lbm_params side_outlet = box(128, 128, 128, LBM_FP32_DEV, LBM_FACE_PRESSURE);
  side_outlet.face[0] = side_outlet.face[1] = LBM_FACE_PRESSURE;
  const Case cases[] = {
      {"blobs_512x512x384_fp32", box(512, 512, 384, LBM_FP32_DEV, LBM_FACE_WALL)},
      {"blobs_512x512x384_fp64", box(512, 512, 384, LBM_FP64, LBM_FACE_WALL)},
      {"periodic_64x8x4_fp16", box(64, 8, 4, LBM_FP16_DEV, LBM_FACE_PERIODIC)},
      {"ragged_96x8x8_fp32", box(96, 8, 8, LBM_FP32_DEV, LBM_FACE_PERIODIC)},
      {"narrow_4x8x8_fp32", box(4, 8, 8, LBM_FP32_DEV, LBM_FACE_PERIODIC)},
      {"short_64x8x3_fp32", box(64, 8, 3, LBM_FP32_DEV, LBM_FACE_PERIODIC)},
      {"outlet_512x512x384_fp32", outlet},
      {"outlets_256x256x256_fp64", box(256, 256, 256, LBM_FP64, LBM_FACE_PRESSURE)},
      {"half_open_256x256x256_fp32", half_open},
      {"side_outlet_128x128x128_fp32", side_outlet},
      {"plane_4096x4096_fp64", box(4096, 4096, 8, LBM_FP64, LBM_FACE_WALL)},
      {"plane_8192x4096_fp32", box(8192, 4096, 4, LBM_FP32_DEV, LBM_FACE_WALL)},
      {"plane_8192x4096_fp64", box(8192, 4096, 4, LBM_FP64, LBM_FACE_WALL)},
      {"plane_8192x8192_fp32", box(8192, 8192, 4, LBM_FP32_DEV, LBM_FACE_WALL)},
      // the largest planes below the 32-bit offset limit and the next row up
      {"limit_5184x5104_fp64", box(5184, 5104, 4, LBM_FP64, LBM_FACE_PERIODIC)},
      {"over_5184x5112_fp64", box(5184, 5112, 4, LBM_FP64, LBM_FACE_PERIODIC)},
      {"limit_7296x7256_fp32", box(7296, 7256, 4, LBM_FP32_DEV, LBM_FACE_PERIODIC)},
      {"over_7296x7264_fp32", box(7296, 7264, 4, LBM_FP32_DEV, LBM_FACE_PERIODIC)},
  };
  for (const Case& c : cases) std::printf("%s %d\n", c.name, lbm::fused_supported(c.p, 8) ? 1 : 0);
  // 16-row tiles: 32/16-bit storage only, ny a multiple of 16
  std::printf("ty16_512x512x384_fp32 %d\n", lbm::fused_supported(box(512, 512, 384, LBM_FP32_DEV, LBM_FACE_WALL), 16));
  std::printf("ty16_512x512x384_fp64 %d\n", lbm::fused_supported(box(512, 512, 384, LBM_FP64, LBM_FACE_WALL), 16));
  std::printf("ty16_64x8x8_fp32 %d\n", lbm::fused_supported(box(64, 8, 8, LBM_FP32_DEV, LBM_FACE_PERIODIC), 16));
  std::printf("ty16_ragged_96x16x8_fp32 %d\n", lbm::fused_supported(box(96, 16, 8, LBM_FP32_DEV, LBM_FACE_PERIODIC), 16));
  // z planes per workgroup chosen by the context
  std::printf("chunk_512x512x384 %d\n", lbm::fused_chunk_planes(512, 512, 384, 8));
  std::printf("chunk_256x256x256 %d\n", lbm::fused_chunk_planes(256, 256, 256, 8));
  std::printf("chunk_128x128x128 %d\n", lbm::fused_chunk_planes(128, 128, 128, 8));
  std::printf("chunk_64x16x24 %d\n", lbm::fused_chunk_planes(64, 16, 24, 8));
  std::printf("chunk_64x8x4 %d\n", lbm::fused_chunk_planes(64, 8, 4, 8));
  return 0;
}
