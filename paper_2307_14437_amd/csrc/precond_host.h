// Host-side pieces of the IC(1) preconditioner setup.
#pragma once

#include <cstdint>
#include <vector>

struct HostTransfer {
  int d = 2, W = 0;
  int64_t nv = 0, n_nodes = 0;
  std::vector<int32_t> elem;       // element of each node or -1
  std::vector<int32_t> elems;      // element vertex ids
  std::vector<double> node_w;      // barycentric weights per node (d+1 each)
  std::vector<int32_t> csc_off, csc_node;
  std::vector<double> csc_w;
  std::vector<uint8_t> bnd;        // 1 = Dirichlet
};

struct HostCsr {
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

bool assemble_pattern_matrix(const HostTransfer& t, const double* T, int npts, HostCsr& A);
void ic_symbolic(const HostCsr& A, int level, std::vector<int64_t>& Lptr, std::vector<int32_t>& Lcol);
bool ic_numeric(const HostCsr& A, double shift, const std::vector<int64_t>& Lptr, const std::vector<int32_t>& Lcol,
                std::vector<double>& Lval);
