#include "layout.hpp"

namespace dmrg {

std::vector<QN> site_phys_qn() { return {site_qn(0), site_qn(1), site_qn(2), site_qn(3)}; }

std::vector<QN> twosite_phys_qn() {
  std::vector<QN> v;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) v.push_back(site_qn(a) + site_qn(b));
  return v;
}

TensorLayout make_tensor_layout(const Bond& l, const Bond& r, const std::vector<QN>& phys_qn) {
  TensorLayout t;
  t.nphys = (int)phys_qn.size();
  t.slab_of_left.assign(l.sec.size(), -1);
  long off = 0;
  for (size_t li = 0; li < l.sec.size(); ++li) {
    Slab s;
    s.li = (int)li;
    s.ml = l.sec[li].dim;
    s.width = 0;
    for (int p = 0; p < (int)phys_qn.size(); ++p) {
      int ri = r.find(l.sec[li].q + phys_qn[p]);
      if (ri < 0) continue;
      s.blocks.push_back({p, ri, r.sec[ri].dim, s.width});
      s.width += r.sec[ri].dim;
    }
    if (s.blocks.empty() || s.ml == 0) continue;
    s.off = off;
    off += (long)s.ml * s.width;
    t.slab_of_left[li] = (int)t.slabs.size();
    t.slabs.push_back(std::move(s));
  }
  t.size = off;
  return t;
}

std::vector<EnvClass> make_env_classes(const Bond& b, const std::vector<QN>& dqs) {
  std::vector<EnvClass> out;
  for (const QN& dq : dqs) {
    EnvClass c;
    c.dq = dq;
    c.block_of_col.assign(b.sec.size(), -1);
    for (size_t ci = 0; ci < b.sec.size(); ++ci) {
      int ri = b.find(b.sec[ci].q + dq);
      if (ri < 0) continue;
      c.block_of_col[ci] = (int)c.blocks.size();
      c.blocks.push_back({ri, (int)ci, b.sec[ri].dim, b.sec[ci].dim, c.nnz});
      c.nnz += (long)b.sec[ri].dim * b.sec[ci].dim;
    }
    out.push_back(std::move(c));
  }
  return out;
}

}  // namespace dmrg
