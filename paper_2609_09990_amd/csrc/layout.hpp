// Block-sparse layouts by (N, 2S_z) quantum numbers.
//
// Bond: sorted list of sectors.  Three-leg tensors (MPS site tensors with 4
// physical states, two-site vectors with 16) are stored slab by slab: for each
// left sector a row-major m_l x W matrix whose column ranges are the blocks of
// the physical states (in order) whose right sector exists.  Environment
// channels are grouped by the quantum-number shift dq of their operator; all
// channels of one class share one block list (row sector = column sector + dq).
#pragma once

#include <map>
#include <vector>

#include "common.hpp"

namespace dmrg {

struct Sector {
  QN q;
  int dim;
};

struct Bond {
  std::vector<Sector> sec;
  int find(QN q) const {
    // sectors are sorted; bonds are short, linear search is fine
    for (size_t i = 0; i < sec.size(); ++i)
      if (sec[i].q == q) return (int)i;
    return -1;
  }
  int total() const {
    int t = 0;
    for (auto& s : sec) t += s.dim;
    return t;
  }
};

struct SlabBlock {
  int phys;   // physical index (0..3 or 0..15)
  int ri;     // right sector index
  int mr;     // right sector dim
  int col0;   // first column inside the slab
};

struct Slab {
  int li;     // left sector index
  int ml;     // rows
  int width;  // columns
  long off;   // element offset of the slab
  std::vector<SlabBlock> blocks;
  int block_of(int phys, int ri) const {
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i].phys == phys && blocks[i].ri == ri) return (int)i;
    return -1;
  }
};

struct TensorLayout {
  std::vector<Slab> slabs;
  std::vector<int> slab_of_left;  // left sector index -> slab index or -1
  long size = 0;
  int nphys = 0;
};

// phys_qn: quantum numbers of the physical states (4 for a site, 16 for two sites).
TensorLayout make_tensor_layout(const Bond& l, const Bond& r, const std::vector<QN>& phys_qn);
std::vector<QN> site_phys_qn();
std::vector<QN> twosite_phys_qn();

struct EnvBlock {
  int ri, ci;   // row / column sector
  int mr, mc;
  long off;     // offset inside one channel's array
};

struct EnvClass {
  QN dq;
  std::vector<EnvBlock> blocks;
  std::vector<int> block_of_col;  // column sector -> block index or -1
  long nnz = 0;
};

// Per-class block lists for a bond, for a given set of shifts.
std::vector<EnvClass> make_env_classes(const Bond& b, const std::vector<QN>& dqs);

}  // namespace dmrg
