// Geometry of one multigrid level in the padded MAC layout, shared by the
// host driver and the gfx950 kernels.
//
// A level is a box of nx*ny*nz cells of edge h surrounded by one layer of
// Dirichlet cells (Section 5 of the paper; label coarsening keeps a box a
// box).  Every field (u_x, u_y, u_z, p) uses the same padded grid of
// (nx+2) x (ny+2) x (nz+2) slots: slot s = I + sy J + sz K, x fastest, with an
// odd row pitch sy and an odd plane pitch sz, so that s & 1 is the parity of
// I + J + K, the red/black colour of the slot.  A field stores its two colours
// apart: slot s lives at element at(s) = (s & 1) half + (s >> 1), so a colour
// pass of the smoothers reads and writes contiguous half-fields.
// Cell (I,J,K) (padded, 1-based for interior cells) owns p at (I,J,K), its
// minus-x face u_x at (I,J,K) and its plus-x face u_x at (I+1,J,K); y and z
// likewise.  Slots that are not unknowns hold zero.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define SG_HD __host__ __device__ __forceinline__
#else
#define SG_HD inline
#endif

struct Geom {
  int nx, ny, nz;   // interior cells
  int sy;           // row pitch (slots), odd
  int sz;           // plane pitch (slots), odd, >= sy * (ny + 2)
  int field;        // elements per field: slots + 8 spare, rounded up to a multiple of 8
  int half;         // field / 2: the colour-1 slots start here
  int rows;         // (ny + 2) * (nz + 2)
  double h, inv_h;  // cell edge and its inverse
  double c;         // eta / h^2 (the viscous stencil weight)
  double eta, gamma;

  SG_HD int idx(int I, int J, int K) const { return I + sy * J + sz * K; }
  // element of slot s inside a field (red/black split)
  SG_HD int at(int s) const { return (s & 1) * half + (s >> 1); }

  // --- unknowns (Section 5: faces between two interior cells, interior cells) ---
  SG_HD bool ux_active(int I, int J, int K) const {
    return I >= 2 && I <= nx && J >= 1 && J <= ny && K >= 1 && K <= nz;
  }
  SG_HD bool uy_active(int I, int J, int K) const {
    return I >= 1 && I <= nx && J >= 2 && J <= ny && K >= 1 && K <= nz;
  }
  SG_HD bool uz_active(int I, int J, int K) const {
    return I >= 1 && I <= nx && J >= 1 && J <= ny && K >= 2 && K <= nz;
  }
  SG_HD bool p_active(int I, int J, int K) const {
    return I >= 1 && I <= nx && J >= 1 && J <= ny && K >= 1 && K <= nz;
  }

  // --- the interior set V2: unknowns not on a cell that touches a Dirichlet cell ---
  SG_HD bool ux_v2(int I, int J, int K) const {
    return I >= 3 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }
  SG_HD bool uy_v2(int I, int J, int K) const {
    return I >= 2 && I <= nx - 1 && J >= 3 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }
  SG_HD bool uz_v2(int I, int J, int K) const {
    return I >= 2 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 3 && K <= nz - 1;
  }
  SG_HD bool p_v2(int I, int J, int K) const {
    return I >= 2 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }
  // red (0) / black (1) class: parity of the 0-based field index, i.e. (I+J+K-3) mod 2
  SG_HD static int parity(int I, int J, int K) { return (I + J + K + 1) & 1; }
  // 8-colour Vanka class of cell (I,J,K): (i&1) + 2(j&1) + 4(k&1), 0-based i,j,k
  SG_HD static int vanka_colour(int I, int J, int K) {
    return ((I - 1) & 1) | (((J - 1) & 1) << 1) | (((K - 1) & 1) << 2);
  }
};

// Offsets of the four fields inside a state vector of 4*field elements.
enum { FUX = 0, FUY = 1, FUZ = 2, FP = 3 };
