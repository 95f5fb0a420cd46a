// Internal layout shared by the gfx950 kernels and the host runtime of liblb.
// Not part of the public interface (include/lb.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

constexpr int NQ = 9;

// One ensemble member as the kernels see it.  Lives in the workspace; every
// field is uniform across a workgroup and read with scalar loads.
struct alignas(256) Member {
    int32_t nx, ny;          // lattice
    int32_t pitch;           // elements per stored row segment (nx rounded up to 64)
    int32_t tiles_x, tiles_y, tile_h;
    int64_t sstride;         // element strides of the population buffer:
    int64_t istride;         //   address of f_i^s(x, y) = s*sstride + i*istride
    int64_t ystride;         //                            + y*ystride + x
    int64_t item_begin;      // first work item of this member in the step launch
    int64_t item_end;
    int32_t tiles_x2, tiles_y2, tile_h2;   // tiles of the two-step pass
    int32_t pad_;
    int64_t item2_begin;     // first work item of this member in the two-step launch
    int64_t item2_end;
    void *f[2];              // ping-pong population buffers, row blocks [y][s][i][pitch]
    double tau[2], itau[2];  // relaxation times and their reciprocals
    double G;                // Shan-Chen coupling
    double g[2][2];          // body acceleration per component
    float shift[2][NQ];      // 16-bit modes: w_i rho0_s; else 0
    float scale[2][NQ];      // 16-bit modes: power-of-two scale; else 1
    float iscale[2][NQ];     // 1 / scale
    float nss[2][NQ];        // -shift * scale (exact: scale is a power of two)
};

// Storage modes (values equal the LB_F64 .. LB_BF16S constants of lb.h).
enum StorageMode { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3 };
enum Forcing { FORCE_SHIFT = 0, FORCE_GUO = 1 };
enum BcY { BC_WALLS = 0, BC_PERIODIC = 1 };

// Outputs of the field (macroscopic) pass: [ny][nx] doubles, any may be null.
struct FieldOut {
    double *rhoA, *rhoB, *ux, *uy;
};

constexpr int RED_NQ = 9;  // per-row partial sums kept by the reduction

}  // namespace lbk
