// Internal data structures of the hpsexp library (host + device).
//
// Solve stage of the hierarchical solver, in this library's notation.
//
// Leaf (one element, p x p nodes, q = p-2): interior nodes i (q*q of them),
// edge nodes e (the non-corner nodes of the element's sides that are not
// on the outer boundary).  With A the collocated operator K - s on the
// interior rows,
//     u_i = W g - S u_e,   W = A_ii^{-1},  S = W A_ie,
//     du/dn on e = T u_e + h,   T = N_e - N_i S,  h = N_i W g,
// where N = [N_e N_i] is the outward normal derivative at the edge nodes.
//
// Merge of boxes a and b (set 1 = a's exterior not shared, 2 = b's, 3 =
// the shared interface): flux continuity on set 3 gives
//     u_3 = -Z [u_ext; g3],   Z = X [B | I],  X = (T_33^a + T_33^b)^{-1},
//     B = [T_31^a | T_32^b],  g3 = h_3^a + h_3^b,
// and the parent's map is
//     T_par = diag(T_11^a, T_22^b) - V X B,   h_par = [h_1^a; h_2^b] - Y g3,
//     V = [T_13^a; T_23^b],   Y = V X.
// Stored per pole: leaf [W | S] (q^2 x (q^2+e)), merge Z (n3 x (ext+n3))
// followed by Y (ext x n3); all complex FP64, column-major.
#pragma once

#include <hip/hip_runtime.h>

namespace hx {

constexpr int kMaxP = 18;
constexpr int kBlock = 256;

struct LeafDesc {
  long long op_off;  // complex offset of [W | S] inside one pole's operator block
  int vec_off;       // offset of the leaf's edge vector in the level-0 h/u arrays
  int e;             // number of edge nodes (non-boundary sides * q)
  int side_mask;     // bit s: side s (0 left, 1 right, 2 bottom, 3 top) is an interface
  int elem;          // element index ex + nex*ey
  int pad;
};

struct BoxDesc {
  long long op_off;  // complex offset of Z (then Y) inside one pole's operator block
  int a_vec, b_vec;  // children's offsets in the level-below h/u arrays
  int vec_off;       // this box's offset in its own level's h/u arrays
  int g3_off;        // offset in this level's g3 array
  int n1, n2, n3;    // exterior-from-a, exterior-from-b, interface sizes
  int idx_off;       // int32 maps: idx1[n1] idx2[n2] idx3a[n3] idx3b[n3]
  int a_box, b_box;  // children's indices in the level below
  int j_off;         // int32 maps ja[n3] jb[n3]: the two element-edge slots
                     // (level-0 vector positions) of each interface node
};

struct PoleCoef {
  double2 alpha;  // pole alpha_m
  double2 cu;     // weight of y_m in the new u: b_m (doubled for m > 0)
  double2 cv;     // weight of y_m in tau * new v: b_m alpha_m (doubled for m > 0)
  // right-hand side of pole m's elliptic solve: g = k1 X1 + k2 X2 + k3 X3
  // with real source fields X (wave: u0, v0; shallow water: eta0, div, curl)
  double2 k1, k2, k3;
  double2 sig;    // shift of the elliptic operator: (alpha/tau)^2, or (a^2 + f^2)/c^2
};

struct SwCoef {   // shallow-water pole sums (doubled for m > 0)
  double2 c0;     // b_m            -> eta'
  double2 c1;     // b_m a_m / s_m  -> E1
  double2 c2;     // b_m / s_m      -> E2
};

}  // namespace hx
