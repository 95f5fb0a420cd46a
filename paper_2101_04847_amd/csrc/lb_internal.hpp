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
    int32_t tiles_x3, tiles_y3, tile_h3;   // tiles of the three-step pass
    int32_t pad3_;
    int64_t item3_begin;     // first work item of this member in the three-step launch
    int64_t item3_end;
    void *f[2];              // ping-pong population buffers, row blocks [y][s][i][pitch]
    double tau[2], itau[2];  // relaxation times and their reciprocals
    double G;                // Shan-Chen coupling
    double g[2][2];          // body acceleration per component
    double aw[2][2];         // Eq. 6 wall acceleration a_s,y of component s on row 0 ([s][0])
                             //   and row ny - 1 ([s][1]); its x part is exactly 0
    int32_t wall_force;      // 1: aw applies (walls and some G_sb != 0)
    int32_t psi_zero;        // 1: psi = 0 on boundary nodes in Eq. 5; 0: psi of the wall row
    int32_t rho_off;         // 16-bit modes: byte offset of the site densities in a row block
    int32_t rho_sstride;     //   and bytes between the two components' density segments
    float scale[2][NQ];      // 16-bit modes: power-of-two scale of the codes; else 1
    float iscale[2][NQ];     // 1 / scale (exact)
    float cscale[3];         // the same scales per weight class (rest, axis, diagonal): they
    float ciscale[3];        //   depend on w_i only; the kernels read these
};

// Storage modes (values equal the LB_F64 .. LB_BF16S constants of lb.h).
enum StorageMode { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3 };
enum Forcing { FORCE_SHIFT = 0, FORCE_GUO = 1 };
// Boundary variant of the step kernels.  BC_WALLS and BC_PERIODIC equal
// LB_WALLS and LB_PERIODIC_Y.  BC_WALLS_WET is the walls variant that also
// reads the Eq. 6 wall force and the psi of boundary nodes from the member
// table; the plain BC_WALLS kernels (neutral walls: no wall force, psi of the
// wall row) keep the registers those terms would cost.
enum BcY { BC_WALLS = 0, BC_PERIODIC = 1, BC_WALLS_WET = 2 };

// Outputs of the field (macroscopic) pass: [ny][nx] doubles, any may be null.
struct FieldOut {
    double *rhoA, *rhoB, *ux, *uy;
};

constexpr int RED_NQ = 9;  // per-row partial sums kept by the reduction

}  // namespace lbk

// Host runtime helpers shared by the 2D and 3D entry points.
namespace lbrt {
// Records the message returned by lb_last_error and returns code.
__attribute__((visibility("hidden"), format(printf, 2, 3))) int32_t fail(int32_t code, const char *fmt, ...);
}  // namespace lbrt

#define HIP_TRY(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return lbrt::fail(LB_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
