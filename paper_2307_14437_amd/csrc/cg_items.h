// Work items of a batched solve: one item per (problem, right-hand side).
//
// Every kernel of a CG iteration runs once per batch with blockIdx.y = item;
// a block reads its item's descriptor (mesh arrays, vector offset, grid
// geometry) and works on that item only.  Problems of one batch share the
// grid shape (d, W, L) and may differ in mesh, box and order s.
#pragma once

#include <hip/hip_runtime.h>

#include "bary.h"

struct CgItem {
  // transfer of the item's problem
  const int* csc_off;
  const int* csc_node;
  const double* csc_w;
  const float* csc_w32;
  const double* imask;        // 1 interior, 0 Dirichlet
  const double* dscale;       // 1 / D_j
  const void* recs;           // ElemRec2 / ElemRec3 per element
  const int* elem;            // element of each grid node or -1
  const int* ell_idx;         // 3D: compact row of each inside node or -1
  const int4* ell_v;          // 3D: vertex ids of the rows
  const double2* ell_w;       // 3D: weights of the rows
  const int4* row32_v;        // 2D: per-node vertex ids (and weight 0) for the FP32 gather
  const float2* row32_w;      // 2D: per-node weights 1 and 2 for the FP32 gather
  const int* rp_meta;         // 2D row-pair form of I^T (int4 per row pair), or null
  const int* rp_tseg;
  const unsigned short* rp_code;
  const float* rp_w32;
  const double* rp_w64;
  const int* rp_dest;
  const int* pv_off;          // partial slots of each vertex
  const int* rp_pos;          // row-pair-major position of each slot
  const int4* seg_row;        // per node: local segments and weights of the FP32 gather through the slots
  const float* seg_row_w2;
  GridGeom g;
  long long nv;               // vertices of the mesh
  long long off;              // offset of the item's vectors in the batch vectors
  int dk;                     // preconditioner: 1 diagonal, 0 none, -1 IC(1)
  int pad;
};
