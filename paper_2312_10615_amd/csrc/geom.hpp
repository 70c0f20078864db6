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
//
// A box padded by Dirichlet cells needs no tables: activity and the V1/V2
// split are arithmetic on (I, J, K).  A domain given by cell labels
// (Section 5: interior, Dirichlet, exterior) carries one 32-bit flag word
// per slot, stored like a field (element at(s)):
//   bits 0-3   u_x, u_y, u_z, p of the slot are unknowns
//   bits 4-7   ... and belong to V2
//   bits 8-16  n_f of u_x, u_y, u_z (3 bits each): the diagonal of A at that
//              face is n_f eta/h^2 (6 except beside exterior cells)
//   bits 17-26 the Vanka local-matrix type of the cell (V1 cells)
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
  const uint32_t* flags;  // labelled domains: flag word per slot (element at(s)); nullptr for a box

  SG_HD int idx(int I, int J, int K) const { return I + sy * J + sz * K; }
  // element of slot s inside a field (red/black split)
  SG_HD int at(int s) const { return (s & 1) * half + (s >> 1); }
  // flag word of slot s (0 outside the field)
  SG_HD uint32_t fw(int s) const { return (unsigned)s < (unsigned)field ? flags[at(s)] : 0u; }
  SG_HD uint32_t fw(int I, int J, int K) const { return fw(idx(I, J, K)); }

  // --- unknowns (Section 5) ---
  SG_HD bool ux_active(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 1u;
    return I >= 2 && I <= nx && J >= 1 && J <= ny && K >= 1 && K <= nz;
  }
  SG_HD bool uy_active(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 2u;
    return I >= 1 && I <= nx && J >= 2 && J <= ny && K >= 1 && K <= nz;
  }
  SG_HD bool uz_active(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 4u;
    return I >= 1 && I <= nx && J >= 1 && J <= ny && K >= 2 && K <= nz;
  }
  SG_HD bool p_active(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 8u;
    return I >= 1 && I <= nx && J >= 1 && J <= ny && K >= 1 && K <= nz;
  }

  // --- the interior set V2: unknowns not on a cell proximal to a Dirichlet or exterior cell ---
  SG_HD bool ux_v2(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 16u;
    return I >= 3 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }
  SG_HD bool uy_v2(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 32u;
    return I >= 2 && I <= nx - 1 && J >= 3 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }
  SG_HD bool uz_v2(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 64u;
    return I >= 2 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 3 && K <= nz - 1;
  }
  SG_HD bool p_v2(int I, int J, int K) const {
    if (flags) return fw(I, J, K) & 128u;
    return I >= 2 && I <= nx - 1 && J >= 2 && J <= ny - 1 && K >= 2 && K <= nz - 1;
  }

  // n_f of velocity component f at slot s (the diagonal of A there is n_f eta/h^2)
  SG_HD int nd(int f, int s) const { return flags ? (int)((fw(s) >> (8 + 3 * f)) & 7u) : 6; }

  // The Vanka subdomain of cell (I,J,K): bit r set when its local face r is an
  // unknown (0/1: u_x minus/plus, 2/3: u_y, 4/5: u_z), and the index of its
  // local inverse in the level's table (for a box: the six bits themselves).
  SG_HD int vface_bits(int I, int J, int K) const {
    if (!flags)
      return (int)(I >= 2) | ((int)(I + 1 <= nx) << 1) | ((int)(J >= 2) << 2) | ((int)(J + 1 <= ny) << 3) |
             ((int)(K >= 2) << 4) | ((int)(K + 1 <= nz) << 5);
    return (int)ux_active(I, J, K) | ((int)ux_active(I + 1, J, K) << 1) | ((int)uy_active(I, J, K) << 2) |
           ((int)uy_active(I, J + 1, K) << 3) | ((int)uz_active(I, J, K) << 4) | ((int)uz_active(I, J, K + 1) << 5);
  }
  SG_HD int vtype(int I, int J, int K, int bits) const {
    return flags ? (int)((fw(I, J, K) >> 17) & 1023u) : bits;
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
