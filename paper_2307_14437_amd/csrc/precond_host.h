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

bool assemble_pattern_matrix(const HostTransfer& t, const double* T, int64_t Wt, int npts, HostCsr& A);
void ic_symbolic(const HostCsr& A, int level, std::vector<int64_t>& Lptr, std::vector<int32_t>& Lcol);
bool ic_numeric(const HostCsr& A, double shift, const std::vector<int64_t>& Lptr, const std::vector<int32_t>& Lcol,
                std::vector<double>& Lval);
// Greedy colouring of the graph of A: vertices in index order, each taking the
// smallest colour no already coloured neighbour has.  Returns the colour count.
int greedy_colouring(const HostCsr& A, std::vector<int32_t>& colour);
// Colouring in Matula and Beck's smallest-last order: vertices removed one at
// a time, each time one of least degree among those left (ties: the smallest
// index), then coloured in the reverse order, each the smallest colour no
// already coloured neighbour has.  Returns the colour count.
int smallest_last_colouring(const HostCsr& A, std::vector<int32_t>& colour);
// B = P A P^T for the order perm (B_ij = A_{perm[i], perm[j]}), rows sorted.
void permute_symmetric(const HostCsr& A, const std::vector<int32_t>& perm, HostCsr& B);
// Drop the off-diagonal entries of a lower pattern that join two vertices of
// the same colour (colour given in the pattern's numbering), except, with
// group given, those inside one group.
void drop_same_colour(const std::vector<int32_t>& colour, std::vector<int64_t>& Lptr, std::vector<int32_t>& Lcol,
                      const std::vector<int32_t>* group = nullptr);
// Blocks of at most `size` vertices: in index order, a vertex not yet in a
// block starts one, which takes not yet placed vertices breadth first (a
// vertex's neighbours in increasing index, rows of A sorted) until full.
// Returns the block count; blk[v] is v's block.
int grow_blocks(const HostCsr& A, int size, std::vector<int32_t>& blk);
// The graph of the blocks: b and c adjacent when A couples a vertex of b to
// one of c (b != c); rows sorted, no self entries.
void block_graph(const HostCsr& A, const std::vector<int32_t>& blk, int nb, HostCsr& G);
