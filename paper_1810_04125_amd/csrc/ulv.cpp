// Host side of the HSS factorization and solve (the method and the kernels
// are in k_ulv.hip).  Per level of the tree, deepest first: the nodes'
// blocks are gathered, transformed by two grouped GEMM launches, and
// LU-factored in 32-column steps (panel kernel, row swaps, two grouped
// GEMMs).  The solve replays the same steps on the right-hand sides.  The
// ranks are known on the host once the compression has ended, so every
// task is built here and uploaded once per call.
#include <chrono>
#include <cstring>

#include "driver.h"

namespace hss {
namespace {

constexpr int UNB = 32;

GemmTask gemm(const double* A, int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, double* C,
              int64_t c_rs, int64_t c_cs, int32_t M, int32_t N, int32_t K, double alpha, double beta) {
  GemmTask t;
  t.A = A; t.a_rs = a_rs; t.a_cs = a_cs;
  t.B = B; t.b_rs = b_rs; t.b_cs = b_cs;
  t.C = C; t.c_rs = c_rs; t.c_cs = c_cs;
  t.M = M; t.N = N; t.K = K; t.pad = 0;
  t.alpha = alpha; t.beta = beta;
  return t;
}

// One launch of the replayed sequence: `count` tasks of one kind from
// offset `off` of that kind's array; a, b: the launch's size caps.
enum Kind { kBuild, kGemm, kPanel, kSwap, kIn, kOut, kSubstF, kSubstB };
struct Launch {
  Kind kind;
  int64_t off;
  int32_t count;
  int64_t a, b;
};

struct Program {
  std::vector<Launch> seq;
  std::vector<GemmTask> gemms;
  std::vector<UlvBuild> builds;
  std::vector<UlvPanel> panels;
  std::vector<UlvSwap> swaps;
  std::vector<UlvMove> moves;
  std::vector<UlvSubst> substs;
  void gemm_launch(const std::vector<GemmTask>& ts) {
    if (ts.empty()) return;
    int64_t M = 1, N = 1;
    for (const GemmTask& t : ts) { M = std::max<int64_t>(M, t.M); N = std::max<int64_t>(N, t.N); }
    seq.push_back(Launch{kGemm, (int64_t)gemms.size(), (int32_t)ts.size(), M, N});
    gemms.insert(gemms.end(), ts.begin(), ts.end());
  }
  template <class T>
  static size_t bytes(const std::vector<T>& v) { return ((sizeof(T) * v.size() + 255) / 256) * 256; }
  size_t device_bytes() const {
    return bytes(gemms) + bytes(builds) + bytes(panels) + bytes(swaps) + bytes(moves) + bytes(substs) + 256;
  }
  // uploads the task arrays into dev (device_bytes() bytes) and launches the sequence on s
  void run(char* dev, int32_t nrhs, int32_t* flag, hipStream_t s) const {
    std::vector<char> host(device_bytes());
    size_t o = 0;
    auto place = [&](const auto& v) {
      const size_t at = o;
      if (!v.empty()) std::memcpy(host.data() + o, v.data(), sizeof(v[0]) * v.size());
      o += bytes(v);
      return at;
    };
    const size_t og = place(gemms), ob = place(builds), op = place(panels), os = place(swaps), om = place(moves);
    const size_t osb = place(substs);
    HSS_HIP_CHECK(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, s));
    HSS_HIP_CHECK(hipStreamSynchronize(s));   // the staging copy is complete before `host` goes
    const GemmTask* g = (const GemmTask*)(dev + og);
    const UlvBuild* b = (const UlvBuild*)(dev + ob);
    const UlvPanel* p = (const UlvPanel*)(dev + op);
    const UlvSwap* w = (const UlvSwap*)(dev + os);
    const UlvMove* mv = (const UlvMove*)(dev + om);
    const UlvSubst* sb = (const UlvSubst*)(dev + osb);
    for (const Launch& L : seq) {
      switch (L.kind) {
        case kBuild: launch_ulv_build(b + L.off, L.count, L.a, s); break;
        case kGemm: launch_gemm(g + L.off, L.count, (int32_t)L.a, (int32_t)L.b, s); break;
        case kPanel: launch_ulv_panel(p + L.off, L.count, flag, s); break;
        case kSwap: launch_ulv_swap(w + L.off, L.count, L.a, s); break;
        case kIn: launch_ulv_rhs_in(mv + L.off, L.count, nrhs, L.a, s); break;
        case kOut: launch_ulv_x_out(mv + L.off, L.count, nrhs, L.a, s); break;
        case kSubstF: launch_ulv_subst(sb + L.off, L.count, nrhs, 0, s); break;
        case kSubstB: launch_ulv_subst(sb + L.off, L.count, nrhs, 1, s); break;
      }
    }
    HSS_HIP_CHECK(hipGetLastError());
  }
};

int32_t nblocks(int32_t k) { return (k + UNB - 1) / UNB; }

// nodes of each level, deepest level first
std::vector<std::vector<int32_t>> by_level(const UlvFactor& f) {
  std::vector<std::vector<int32_t>> L(f.maxlevel + 1);
  for (int32_t v = 0; v < (int32_t)f.nodes.size(); ++v) L[f.nodes[v].level].push_back(v);
  return L;
}

}  // namespace

void ulv_factor(hss_matrix* h) {
  Job& J = *h->job;
  const Problem& P = J.probs[h->k];
  if ((int32_t)J.ulv.size() < (int32_t)J.probs.size()) J.ulv.resize(J.probs.size());
  if (J.ulv[h->k]) return;   // factored already
  const auto t0 = std::chrono::steady_clock::now();
  auto F = std::make_unique<UlvFactor>();
  UlvFactor& f = *F;
  const int32_t nn = P.nn;
  f.nodes.resize(nn);
  for (int32_t v = 0; v < nn; ++v) {
    const int32_t g = P.node0 + v;
    const NodeDesc& d = J.desc[g];
    const NodeState& st = J.st_h[g];
    UlvFactor::Node& n = f.nodes[v];
    n.g = g;
    n.level = d.level;
    n.leaf = d.leaf;
    n.lo = d.lo;
    n.left = d.left < 0 ? -1 : d.left - P.node0;
    n.right = d.right < 0 ? -1 : d.right - P.node0;
    f.maxlevel = std::max(f.maxlevel, d.level);
    if (d.parent >= 0 && st.rank[0] != st.rank[1])
      throw Error(HSS_ERR_INVALID_ARG, "node " + std::to_string(v) + " has row rank " + std::to_string(st.rank[0]) +
                                           " and column rank " + std::to_string(st.rank[1]) +
                                           "; the factorization needs equal ranks");
  }
  // local sizes bottom-up: a leaf's rows, above the children's ranks
  for (int32_t v = nn - 1; v >= 0; --v) {
    UlvFactor::Node& n = f.nodes[v];
    const NodeDesc& d = J.desc[n.g];
    if (n.leaf) n.m = d.hi - d.lo;
    else {
      n.rl = f.nodes[n.left].r;
      n.m = f.nodes[n.left].r + f.nodes[n.right].r;
    }
    if (d.parent < 0) {
      n.r = 0;
      n.k = n.m;
    } else {
      const NodeState& st = J.st_h[n.g];
      n.r = st.rank[0];
      n.k = n.m - n.r;
      if (st.m[0] != n.m || st.m[1] != n.m)
        throw Error(HSS_ERR_INTERNAL, "node " + std::to_string(v) + ": local size differs from its children's ranks");
      n.Jr = J.ipool + d.J[0];
      n.Jc = J.ipool + d.J[1];
      n.Er = J.epool + d.E[0];
      n.Ec = J.epool + d.E[1];
      n.eldr = d.eld[0];
      n.eldc = d.eld[1];
    }
  }
  int64_t ftot = 0, itot = 0, ptot = 0;
  for (UlvFactor::Node& n : f.nodes) {
    n.F = ftot;
    ftot += ((int64_t)n.m * n.m + 31) / 32 * 32;
    n.inv = itot;
    itot += (int64_t)nblocks(n.k) * 2 * UNB * UNB;
    n.piv = ptot;
    ptot += (n.k + 7) / 8 * 8;
    n.Y = f.ytot;
    f.ytot += n.m;
  }
  f.fpool = (double*)J.dalloc(sizeof(double) * std::max<int64_t>(ftot, 1));
  f.ipool = (double*)J.dalloc(sizeof(double) * std::max<int64_t>(itot, 1));
  f.ppool = (int32_t*)J.dalloc(sizeof(int32_t) * std::max<int64_t>(ptot, 1));
  f.fbytes = 8 * (ftot + itot) + 4 * ptot;

  Program prog;
  const auto levels = by_level(f);
  for (int lev = f.maxlevel; lev >= 0; --lev) {
    const std::vector<int32_t>& L = levels[lev];
    if (L.empty()) continue;
    // gather
    int64_t maxe = 1;
    const int64_t b0 = (int64_t)prog.builds.size();
    for (int32_t v : L) {
      const UlvFactor::Node& n = f.nodes[v];
      const NodeDesc& d = J.desc[n.g];
      UlvBuild b{};
      b.F = f.fpool + n.F;
      b.m = n.m; b.k = n.k; b.r = n.r;
      b.Jr = n.Jr; b.Jc = n.Jc;
      if (n.leaf) {
        b.D = J.dpool + d.D;
      } else {
        const UlvFactor::Node& l = f.nodes[n.left];
        const UlvFactor::Node& r = f.nodes[n.right];
        b.Fl = f.fpool + l.F; b.kl = l.k; b.ml = l.m;
        b.Fr = f.fpool + r.F; b.kr = r.k; b.mr = r.m;
        b.rl = n.rl;
        b.B12 = J.epool + d.B12; b.ld12 = d.b12ld;
        b.B21 = J.epool + d.B21; b.ld21 = d.b21ld;
      }
      prog.builds.push_back(b);
      maxe = std::max<int64_t>(maxe, (int64_t)n.m * n.m);
    }
    prog.seq.push_back(Launch{kBuild, b0, (int32_t)L.size(), maxe, 0});
    // Dhat = T_r D' T_c^T: {F_SR -= F_SS E_c, F_RR -= F_RS E_c}, then
    // {F_RR -= E_r^T F_SR, F_RS -= E_r^T F_SS}
    std::vector<GemmTask> g1, g2;
    for (int32_t v : L) {
      const UlvFactor::Node& n = f.nodes[v];
      if (n.Jr == nullptr || n.k == 0 || n.r == 0) continue;
      double* Fm = f.fpool + n.F;
      const int64_t m = n.m, k = n.k;
      double* FRR = Fm;
      double* FRS = Fm + k * m;
      double* FSR = Fm + k;
      double* FSS = Fm + k + k * m;
      g1.push_back(gemm(FSS, 1, m, n.Ec, 1, n.eldc, FSR, 1, m, n.r, n.k, n.r, -1.0, 1.0));
      g1.push_back(gemm(FRS, 1, m, n.Ec, 1, n.eldc, FRR, 1, m, n.k, n.k, n.r, -1.0, 1.0));
      g2.push_back(gemm(n.Er, n.eldr, 1, FSR, 1, m, FRR, 1, m, n.k, n.k, n.r, -1.0, 1.0));
      g2.push_back(gemm(n.Er, n.eldr, 1, FSS, 1, m, FRS, 1, m, n.k, n.r, n.r, -1.0, 1.0));
    }
    prog.gemm_launch(g1);
    prog.gemm_launch(g2);
    // blocked LU of the first k columns
    int32_t nsteps = 0;
    for (int32_t v : L) nsteps = std::max(nsteps, nblocks(f.nodes[v].k));
    for (int32_t st = 0; st < nsteps; ++st) {
      const int32_t jb = st * UNB;
      const int64_t p0 = (int64_t)prog.panels.size(), s0 = (int64_t)prog.swaps.size();
      int64_t maxcols = 0;
      std::vector<GemmTask> u12, upd;
      for (int32_t v : L) {
        const UlvFactor::Node& n = f.nodes[v];
        if (n.k <= jb) continue;
        const int32_t nb = std::min(UNB, n.k - jb);
        double* Fm = f.fpool + n.F;
        const int64_t m = n.m;
        double* inv = f.ipool + n.inv + (int64_t)st * 2 * UNB * UNB;
        prog.panels.push_back(UlvPanel{Fm, inv, f.ppool + n.piv, n.m, n.k, jb, nb});
        const int64_t c0 = jb + nb;
        if (c0 < m) {
          prog.swaps.push_back(UlvSwap{Fm, f.ppool + n.piv, m, c0, m, jb, nb});
          maxcols = std::max<int64_t>(maxcols, m - c0);
          // U12 = Linv A12 (in place: K = nb fits one K tile, so each output
          // tile has read its inputs before it is written), A22 -= L21 U12
          double* A12 = Fm + jb + c0 * m;
          u12.push_back(gemm(inv, 1, UNB, A12, 1, m, A12, 1, m, nb, (int32_t)(m - c0), nb, 1.0, 0.0));
          upd.push_back(gemm(Fm + c0 + (int64_t)jb * m, 1, m, A12, 1, m, Fm + c0 + c0 * m, 1, m, (int32_t)(m - c0),
                             (int32_t)(m - c0), nb, -1.0, 1.0));
        }
      }
      prog.seq.push_back(Launch{kPanel, p0, (int32_t)(prog.panels.size() - p0), 0, 0});
      if ((int64_t)prog.swaps.size() > s0) prog.seq.push_back(Launch{kSwap, s0, (int32_t)(prog.swaps.size() - s0), maxcols, 0});
      prog.gemm_launch(u12);
      prog.gemm_launch(upd);
    }
  }
  char* dev = (char*)J.dalloc(prog.device_bytes());
  int32_t* flag = (int32_t*)J.dalloc(sizeof(int32_t));
  HSS_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int32_t), J.stream));
  prog.run(dev, 0, flag, J.stream);
  int32_t bad = 0;
  HSS_HIP_CHECK(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, J.stream));
  HSS_HIP_CHECK(hipStreamSynchronize(J.stream));
  J.drop(dev);
  J.drop(flag);
  if (bad) {
    J.drop(f.fpool);
    J.drop(f.ipool);
    J.drop(f.ppool);
    throw Error(HSS_ERR_SINGULAR, "a zero pivot: the compressed matrix (or a node's redundant block) is singular");
  }
  f.factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  J.ulv[h->k] = std::move(F);
}

namespace {
Program solve_program(const UlvFactor& f, int32_t nrhs, const double* Bp, double* Xp, int64_t n, double* Y) {
  Program prog;
  const auto levels = by_level(f);
  auto Yof = [&](const UlvFactor::Node& q) { return Y + q.Y * nrhs; };
  // few right-hand sides: one fused substitution launch per level and pass
  const bool fused = nrhs <= UST_MAXR;
  // forward, deepest level first
  for (int lev = f.maxlevel; lev >= 0; --lev) {
    const std::vector<int32_t>& L = levels[lev];
    if (L.empty()) continue;
    const int64_t m0 = (int64_t)prog.moves.size();
    int64_t maxe = 1;
    std::vector<GemmTask> tr;
    for (int32_t v : L) {
      const UlvFactor::Node& q = f.nodes[v];
      UlvMove mv{};
      mv.Y = Yof(q);
      mv.J = q.Jr;
      mv.m = q.m; mv.k = q.k; mv.r = q.r;
      if (q.leaf) {
        mv.ext = const_cast<double*>(Bp);
        mv.ldext = n;
        mv.lo = q.lo;
      } else {
        const UlvFactor::Node& l = f.nodes[q.left];
        const UlvFactor::Node& r = f.nodes[q.right];
        mv.Yl = Yof(l); mv.kl = l.k; mv.ml = l.m;
        mv.Yr = Yof(r); mv.kr = r.k; mv.mr = r.m;
        mv.rl = q.rl;
      }
      prog.moves.push_back(mv);
      maxe = std::max<int64_t>(maxe, q.m);
      if (q.Jr && q.k > 0 && q.r > 0)   // b_R -= E_r^T b_S
        tr.push_back(gemm(q.Er, q.eldr, 1, Yof(q) + q.k, 1, q.m, Yof(q), 1, q.m, q.k, nrhs, q.r, -1.0, 1.0));
    }
    prog.seq.push_back(Launch{kIn, m0, (int32_t)L.size(), maxe, 0});
    prog.gemm_launch(tr);
    if (fused) {
      prog.seq.push_back(Launch{kSubstF, (int64_t)prog.substs.size(), (int32_t)L.size(), 0, 0});
      for (int32_t v : L) {
        const UlvFactor::Node& q = f.nodes[v];
        prog.substs.push_back(UlvSubst{Yof(q), f.fpool + q.F, f.ipool + q.inv, f.ppool + q.piv, q.m, q.k});
      }
      continue;
    }
    int32_t nsteps = 0;
    for (int32_t v : L) nsteps = std::max(nsteps, nblocks(f.nodes[v].k));
    for (int32_t st = 0; st < nsteps; ++st) {
      const int32_t jb = st * UNB;
      const int64_t s0 = (int64_t)prog.swaps.size();
      std::vector<GemmTask> dl, up;
      for (int32_t v : L) {
        const UlvFactor::Node& q = f.nodes[v];
        if (q.k <= jb) continue;
        const int32_t nb = std::min(UNB, q.k - jb);
        const int64_t m = q.m;
        double* Yq = Yof(q);
        const double* Fm = f.fpool + q.F;
        const double* inv = f.ipool + q.inv + (int64_t)st * 2 * UNB * UNB;
        prog.swaps.push_back(UlvSwap{Yq, f.ppool + q.piv, m, 0, nrhs, jb, nb});
        dl.push_back(gemm(inv, 1, UNB, Yq + jb, 1, m, Yq + jb, 1, m, nb, nrhs, nb, 1.0, 0.0));   // y_j = Linv y_j
        if (jb + nb < m)
          up.push_back(gemm(Fm + (jb + nb) + (int64_t)jb * m, 1, m, Yq + jb, 1, m, Yq + jb + nb, 1, m,
                            (int32_t)(m - jb - nb), nrhs, nb, -1.0, 1.0));
      }
      prog.seq.push_back(Launch{kSwap, s0, (int32_t)(prog.swaps.size() - s0), nrhs, 0});
      prog.gemm_launch(dl);
      prog.gemm_launch(up);
    }
  }
  // backward, root first
  for (int lev = 0; lev <= f.maxlevel; ++lev) {
    const std::vector<int32_t>& L = levels[lev];
    if (L.empty()) continue;
    std::vector<GemmTask> urs;
    int32_t nsteps = 0;
    for (int32_t v : L) {
      const UlvFactor::Node& q = f.nodes[v];
      nsteps = std::max(nsteps, nblocks(q.k));
      if (q.r > 0 && q.k > 0)   // y_R -= U_RS x_S
        urs.push_back(gemm(f.fpool + q.F + (int64_t)q.k * q.m, 1, q.m, Yof(q) + q.k, 1, q.m, Yof(q), 1, q.m, q.k,
                           nrhs, q.r, -1.0, 1.0));
    }
    prog.gemm_launch(urs);
    if (fused) {
      prog.seq.push_back(Launch{kSubstB, (int64_t)prog.substs.size(), (int32_t)L.size(), 0, 0});
      for (int32_t v : L) {
        const UlvFactor::Node& q = f.nodes[v];
        prog.substs.push_back(UlvSubst{Yof(q), f.fpool + q.F, f.ipool + q.inv, f.ppool + q.piv, q.m, q.k});
      }
      nsteps = 0;
    }
    for (int32_t st = nsteps - 1; st >= 0; --st) {
      const int32_t jb = st * UNB;
      std::vector<GemmTask> di, ab;
      for (int32_t v : L) {
        const UlvFactor::Node& q = f.nodes[v];
        if (q.k <= jb) continue;
        const int32_t nb = std::min(UNB, q.k - jb);
        const int64_t m = q.m;
        double* Yq = Yof(q);
        const double* inv = f.ipool + q.inv + (int64_t)st * 2 * UNB * UNB + UNB * UNB;
        di.push_back(gemm(inv, 1, UNB, Yq + jb, 1, m, Yq + jb, 1, m, nb, nrhs, nb, 1.0, 0.0));   // x_j = Uinv y_j
        if (jb > 0)
          ab.push_back(gemm(f.fpool + q.F + (int64_t)jb * m, 1, m, Yq + jb, 1, m, Yq, 1, m, jb, nrhs, nb, -1.0, 1.0));
      }
      prog.gemm_launch(di);
      prog.gemm_launch(ab);
    }
    std::vector<GemmTask> ec;
    const int64_t m0 = (int64_t)prog.moves.size();
    int64_t maxe = 1;
    for (int32_t v : L) {
      const UlvFactor::Node& q = f.nodes[v];
      if (q.Jc && q.k > 0 && q.r > 0)   // x_S -= E_c x_R
        ec.push_back(gemm(q.Ec, 1, q.eldc, Yof(q), 1, q.m, Yof(q) + q.k, 1, q.m, q.r, nrhs, q.k, -1.0, 1.0));
      UlvMove mv{};
      mv.Y = Yof(q);
      mv.J = q.Jc;
      mv.m = q.m; mv.k = q.k; mv.r = q.r;
      if (q.leaf) {
        mv.ext = Xp;
        mv.ldext = n;
        mv.lo = q.lo;
      } else {
        const UlvFactor::Node& l = f.nodes[q.left];
        const UlvFactor::Node& r = f.nodes[q.right];
        mv.Yl = Yof(l); mv.kl = l.k; mv.ml = l.m;
        mv.Yr = Yof(r); mv.kr = r.k; mv.mr = r.m;
        mv.rl = q.rl;
      }
      prog.moves.push_back(mv);
      maxe = std::max<int64_t>(maxe, q.m);
    }
    prog.gemm_launch(ec);
    prog.seq.push_back(Launch{kOut, m0, (int32_t)L.size(), maxe, 0});
  }
  return prog;
}
}  // namespace

void ulv_solve_permuted(const hss_matrix* h, int32_t nrhs, const double* Bp, double* Xp, hipStream_t s) {
  const Job& J = *h->job;
  if ((int32_t)J.ulv.size() <= h->k || !J.ulv[h->k])
    throw Error(HSS_ERR_INVALID_ARG, "the matrix is not factored (call hss_factor first)");
  const UlvFactor& f = *J.ulv[h->k];
  const Problem& P = J.probs[h->k];
  double* Y = nullptr;
  HSS_HIP_CHECK(hipMallocAsync((void**)&Y, sizeof(double) * std::max<int64_t>(f.ytot * nrhs, 1), s));
  Program prog = solve_program(f, nrhs, Bp, Xp, P.n, Y);
  char* dev = nullptr;
  HSS_HIP_CHECK(hipMallocAsync((void**)&dev, prog.device_bytes(), s));
  prog.run(dev, nrhs, nullptr, s);
  HSS_HIP_CHECK(hipFreeAsync(dev, s));
  HSS_HIP_CHECK(hipFreeAsync(Y, s));
}

}  // namespace hss
