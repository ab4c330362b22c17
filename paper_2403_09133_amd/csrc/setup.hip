// lorads_setup: validation, structure detection and device layouts.
#include <algorithm>
#include <numeric>

#include "problem.hpp"

namespace lorads {

[[noreturn]] void fail(lorads_status s, const std::string& msg) { throw Error{s, msg}; }

namespace {

void check(bool ok, const std::string& msg) {
  if (!ok) fail(LORADS_EINVAL, msg);
}

// counting-sort style CSR build: keys in [0, nrows)
void csr_counts(const std::vector<int>& key, int nrows, std::vector<int>& ptr) {
  ptr.assign(nrows + 1, 0);
  for (int k : key) ptr[k + 1]++;
  for (int i = 0; i < nrows; ++i) ptr[i + 1] += ptr[i];
}

}  // namespace

void validate(const lorads_problem& p) {
  check(p.n >= 1, "n must be >= 1");
  check(p.m >= 1, "m must be >= 1");
  check(p.a_nnz >= 1, "a_nnz must be >= 1");
  check(p.c_nnz >= 0, "c_nnz must be >= 0");
  check(p.a_nnz < (int64_t)INT32_MAX / 2 && p.c_nnz < (int64_t)INT32_MAX / 2,
        "too many triplets for 32-bit offsets");
  check(p.a_con && p.a_row && p.a_col && p.a_val && p.b, "null constraint arrays");
  check(p.c_nnz == 0 || (p.c_row && p.c_col && p.c_val), "null cost arrays");
  const int n = p.n, m = p.m;
  for (int64_t e = 0; e < p.c_nnz; ++e) {
    check(p.c_row[e] >= 0 && p.c_col[e] < n && p.c_row[e] <= p.c_col[e],
          "cost triplet " + std::to_string(e) + " out of range or below the diagonal");
    check(std::isfinite(p.c_val[e]), "non-finite cost value");
  }
  std::vector<int> cnt(m, 0);
  for (int64_t e = 0; e < p.a_nnz; ++e) {
    check(p.a_con[e] >= 0 && p.a_con[e] < m, "constraint id out of range at triplet " + std::to_string(e));
    check(p.a_row[e] >= 0 && p.a_col[e] < n && p.a_row[e] <= p.a_col[e],
          "constraint triplet " + std::to_string(e) + " out of range or below the diagonal");
    check(std::isfinite(p.a_val[e]), "non-finite constraint value");
    cnt[p.a_con[e]]++;
  }
  for (int i = 0; i < m; ++i) check(cnt[i] > 0, "constraint " + std::to_string(i) + " has no triplet");
  for (int i = 0; i < m; ++i) check(std::isfinite(p.b[i]), "non-finite b");
  check(std::isfinite(p.mu) && p.mu >= 0.0, "mu must be finite and >= 0 (a convex objective)");
}

std::unique_ptr<Problem> ingest(const lorads_problem& p, hipStream_t s) {
  validate(p);
  const int n = p.n, m = p.m;
  std::vector<int> cnt(m, 0);
  for (int64_t e = 0; e < p.a_nnz; ++e) cnt[p.a_con[e]]++;

  auto P = std::make_unique<Problem>();
  P->n = n;
  P->mu = p.mu;
  P->m = m;
  P->a_nnz = p.a_nnz;
  P->c_nnz = p.c_nnz;

  // ---------------- norms ----------------
  for (int i = 0; i < m; ++i) {
    const double a = std::fabs(p.b[i]);
    P->b_inf = std::max(P->b_inf, a);
    P->b_1 += a;
    P->b_2 += p.b[i] * p.b[i];
  }
  P->b_2 = std::sqrt(P->b_2);
  {
    // C as the full symmetric matrix: merge duplicates before the norms
    std::vector<std::pair<int64_t, double>> ent;
    ent.reserve(p.c_nnz);
    for (int64_t e = 0; e < p.c_nnz; ++e)
      ent.push_back({(int64_t)p.c_row[e] * n + p.c_col[e], p.c_val[e]});
    std::sort(ent.begin(), ent.end(),
              [](const auto& a, const auto& b) { return a.first < b.first; });
    double fro = 0, l1 = 0;
    for (size_t i = 0; i < ent.size();) {
      size_t j = i;
      double v = 0;
      while (j < ent.size() && ent[j].first == ent[i].first) v += ent[j++].second;
      const int64_t key = ent[i].first;
      const double mult = (key / n == key % n) ? 1.0 : 2.0;
      fro += mult * v * v;
      l1 += mult * std::fabs(v);
      i = j;
    }
    P->c_fro = std::sqrt(fro);
    P->c_1 = l1;
  }

  // ---------------- structure detection ----------------
  // first triplet of each constraint
  std::vector<int64_t> first(m, -1);
  for (int64_t e = 0; e < p.a_nnz; ++e)
    if (first[p.a_con[e]] < 0) first[p.a_con[e]] = e;
  bool diag = true, pair = true;
  for (int i = 0; i < m && (diag || pair); ++i) {
    if (cnt[i] != 1) { diag = pair = false; break; }
    const int64_t e = first[i];
    if (p.a_row[e] != p.a_col[e]) diag = false;
    if (p.a_row[e] == p.a_col[e]) pair = false;
  }
  P->structure = diag ? LORADS_STRUCT_DIAG : (pair ? LORADS_STRUCT_PAIR : LORADS_STRUCT_GENERIC);

  // ---------------- internal constraint order ----------------
  std::vector<int> perm(m);
  std::iota(perm.begin(), perm.end(), 0);
  if (P->structure == LORADS_STRUCT_DIAG) {
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      return p.a_row[first[a]] < p.a_row[first[b]];
    });
  } else if (P->structure == LORADS_STRUCT_PAIR) {
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      const int64_t ea = first[a], eb = first[b];
      if (p.a_row[ea] != p.a_row[eb]) return p.a_row[ea] < p.a_row[eb];
      return p.a_col[ea] < p.a_col[eb];
    });
  }
  P->perm_identity = true;
  for (int i = 0; i < m; ++i)
    if (perm[i] != i) { P->perm_identity = false; break; }
  std::vector<int> iperm(m);
  for (int i = 0; i < m; ++i) iperm[perm[i]] = i;

  std::vector<double> b_int(m);
  for (int i = 0; i < m; ++i) b_int[i] = p.b[perm[i]];

  // ---------------- constraint-CSR (internal order) ----------------
  // (RANK1 is decided after it: it needs each constraint's merged triplets)
  std::vector<int> kcon(p.a_nnz);
  for (int64_t e = 0; e < p.a_nnz; ++e) kcon[e] = iperm[p.a_con[e]];
  std::vector<int> kptr;
  csr_counts(kcon, m, kptr);
  std::vector<int> krow(p.a_nnz), kcol(p.a_nnz);
  std::vector<double> kval(p.a_nnz);
  {
    std::vector<int> pos(kptr.begin(), kptr.end() - 1);
    for (int64_t e = 0; e < p.a_nnz; ++e) {
      const int q = pos[kcon[e]]++;
      krow[q] = p.a_row[e];
      kcol[q] = p.a_col[e];
      kval[q] = p.a_val[e];
    }
  }
  // ---------------- RANK1: every A_i = c_i a_i a_i^T ----------------
  if (P->structure == LORADS_STRUCT_GENERIC) {
    std::vector<int> r1ptr(1, 0), r1idx;
    std::vector<double> r1val, r1c;
    bool rank1 = true;
    std::vector<std::pair<int64_t, double>> ent;
    std::vector<int> sup;
    std::vector<double> dg, a;
    for (int i = 0; i < m && rank1; ++i) {
      // merged triplets of A_i, keyed (row, col) with row <= col
      ent.clear();
      for (int q = kptr[i]; q < kptr[i + 1]; ++q) ent.push_back({(int64_t)krow[q] * n + kcol[q], kval[q]});
      std::sort(ent.begin(), ent.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      size_t w = 0;
      for (size_t q = 0; q < ent.size(); ++q) {
        if (w > 0 && ent[w - 1].first == ent[q].first) ent[w - 1].second += ent[q].second;
        else ent[w++] = ent[q];
      }
      ent.resize(w);
      sup.clear();
      for (const auto& e : ent) { sup.push_back((int)(e.first / n)); sup.push_back((int)(e.first % n)); }
      std::sort(sup.begin(), sup.end());
      sup.erase(std::unique(sup.begin(), sup.end()), sup.end());
      const size_t k = sup.size();
      // every pair of the support must be present: a_j a_k != 0 for nonzero a
      if (ent.size() != k * (k + 1) / 2) { rank1 = false; break; }
      auto find = [&](int j, int l) -> double {
        const int64_t key = (int64_t)std::min(j, l) * n + std::max(j, l);
        auto it = std::lower_bound(ent.begin(), ent.end(), key,
                                   [](const auto& x, int64_t v) { return x.first < v; });
        return (it != ent.end() && it->first == key) ? it->second : 0.0;
      };
      dg.assign(k, 0.0);
      size_t piv = 0;
      for (size_t t = 0; t < k; ++t) {
        dg[t] = find(sup[t], sup[t]);
        if (std::fabs(dg[t]) > std::fabs(dg[piv])) piv = t;
      }
      const double c = dg[piv] > 0 ? 1.0 : -1.0;
      a.assign(k, 0.0);
      for (size_t t = 0; t < k && rank1; ++t) {
        if (!(dg[t] * c > 0)) { rank1 = false; break; }
        a[t] = std::sqrt(dg[t] * c);
        if (t != piv && c * find(sup[piv], sup[t]) < 0) a[t] = -a[t];
      }
      for (size_t t = 0; t < k && rank1; ++t)
        for (size_t u = t + 1; u < k; ++u) {
          const double want = c * a[t] * a[u], got = find(sup[t], sup[u]);
          if (std::fabs(got - want) > 1e-12 * std::max(std::fabs(got), std::fabs(want))) { rank1 = false; break; }
        }
      if (!rank1) break;
      for (size_t t = 0; t < k; ++t) { r1idx.push_back(sup[t]); r1val.push_back(a[t]); }
      r1ptr.push_back((int)r1idx.size());
      r1c.push_back(c);
    }
    if (rank1) {
      P->structure = LORADS_STRUCT_RANK1;
      std::vector<int> scon, sstart, cseg(1, 0);
      for (int i = 0; i < m; ++i) {
        for (int e = r1ptr[i]; e < r1ptr[i + 1]; e += kR1Seg) {
          scon.push_back(i);
          sstart.push_back(e);
        }
        cseg.push_back((int)scon.size());
      }
      sstart.push_back(r1ptr[m]);
      std::vector<int> tkey(r1idx.begin(), r1idx.end()), tptr;
      csr_counts(tkey, n, tptr);
      std::vector<int> tcon(r1idx.size());
      std::vector<double> tval(r1idx.size());
      std::vector<int> pos(tptr.begin(), tptr.end() - 1);
      for (int i = 0; i < m; ++i)
        for (int e = r1ptr[i]; e < r1ptr[i + 1]; ++e) {
          const int t = pos[r1idx[e]]++;
          tcon[t] = i;
          tval[t] = r1val[e];
        }
      P->r1ptr.upload(r1ptr, s);
      P->r1idx.upload(r1idx, s);
      P->r1val.upload(r1val, s);
      P->r1c.upload(r1c, s);
      P->r1scon.upload(scon, s);
      P->r1sstart.upload(sstart, s);
      P->r1cseg.upload(cseg, s);
      P->r1tptr.upload(tptr, s);
      P->r1tcon.upload(tcon, s);
      P->r1tval.upload(tval, s);
      std::vector<float> f1(r1val.begin(), r1val.end()), f2(r1c.begin(), r1c.end()),
          f3(tval.begin(), tval.end());
      P->r1valf.upload(f1, s);
      P->r1cf.upload(f2, s);
      P->r1tvalf.upload(f3, s);
      P->r1nseg = (int)scon.size();
    }
  }
  // ---------------- adjoint row-CSR ----------------
  {
    std::vector<int> rkey;
    rkey.reserve(2 * p.a_nnz);
    for (int64_t e = 0; e < p.a_nnz; ++e) {
      rkey.push_back(p.a_row[e]);
      if (p.a_row[e] != p.a_col[e]) rkey.push_back(p.a_col[e]);
    }
    std::vector<int> aptr;
    csr_counts(rkey, n, aptr);
    const size_t na = rkey.size();
    std::vector<int> acol(na), acon(na);
    std::vector<double> aval(na);
    std::vector<int> pos(aptr.begin(), aptr.end() - 1);
    // iterate in internal constraint order so rows list constraints ascending
    for (int i = 0; i < m; ++i) {
      for (int q = kptr[i]; q < kptr[i + 1]; ++q) {
        const int j = krow[q], k = kcol[q];
        int t = pos[j]++;
        acol[t] = k; acon[t] = i; aval[t] = kval[q];
        if (j != k) {
          t = pos[k]++;
          acol[t] = j; acon[t] = i; aval[t] = kval[q];
        }
      }
    }
    P->aptr.upload(aptr, s);
    P->acol.upload(acol, s);
    P->acon.upload(acon, s);
    P->aval.upload(aval, s);
    std::vector<float> af(aval.begin(), aval.end());
    P->avalf.upload(af, s);
  }
  // ---------------- C row-CSR ----------------
  {
    std::vector<int> rkey;
    rkey.reserve(2 * p.c_nnz);
    for (int64_t e = 0; e < p.c_nnz; ++e) {
      rkey.push_back(p.c_row[e]);
      if (p.c_row[e] != p.c_col[e]) rkey.push_back(p.c_col[e]);
    }
    std::vector<int> cptr;
    csr_counts(rkey, n, cptr);
    const size_t nc = rkey.size();
    std::vector<int> ccol(nc);
    std::vector<double> cval(nc);
    std::vector<int> pos(cptr.begin(), cptr.end() - 1);
    for (int64_t e = 0; e < p.c_nnz; ++e) {
      const int j = p.c_row[e], k = p.c_col[e];
      int t = pos[j]++;
      ccol[t] = k; cval[t] = p.c_val[e];
      if (j != k) {
        t = pos[k]++;
        ccol[t] = j; cval[t] = p.c_val[e];
      }
    }
    P->cptr.upload(cptr, s);
    if (nc) {
      P->ccol.upload(ccol, s);
      P->cval.upload(cval, s);
      std::vector<float> cf(cval.begin(), cval.end());
      P->cvalf.upload(cf, s);
    }
    // a diagonal C (at most one entry per row, on the diagonal): its entries
    // by row, so (C D)_j = c_j D_j can be formed where it is used
    bool cdiag = true;
    for (int j = 0; j < n && cdiag; ++j) {
      const int cnt = cptr[j + 1] - cptr[j];
      if (cnt > 1 || (cnt == 1 && ccol[cptr[j]] != j)) cdiag = false;
    }
    if (cdiag) {
      std::vector<double> cd(n, 0.0);
      for (int j = 0; j < n; ++j)
        if (cptr[j + 1] > cptr[j]) cd[j] = cval[cptr[j]];
      P->cdiag.upload(cd, s);
    }
    // a dense C (a quarter of the entries or more) is also kept dense, for
    // the matrix-core products
    if (n >= kDenseCMinN && n <= 32768 && (double)nc >= 0.25 * (double)n * n) {
      // tile-major: the 16 x 64 tile of rows 16 t .. 16 t + 15 and columns
      // 64 b .. 64 b + 63 is one contiguous run of 1024 entries (row-major
      // inside), the tiles of a row band in column order; entries past n are zero
      const int ldc = (n + 63) / 64 * 64;
      const size_t bands = (size_t)(n + 15) / 16, kb = (size_t)ldc / 64;
      std::vector<double> cdn(bands * 16 * ldc, 0.0);
      for (int j = 0; j < n; ++j)
        for (int e = cptr[j]; e < cptr[j + 1]; ++e) {
          const size_t c = (size_t)ccol[e];
          cdn[(((size_t)(j / 16) * kb + c / 64) * 16 + (size_t)(j % 16)) * 64 + c % 64] += cval[e];
        }
      std::vector<float> cdf(cdn.begin(), cdn.end());
      P->cdense.upload(cdn, s);
      P->cdensef.upload(cdf, s);
      P->ldc = ldc;
    }
  }

  // ---------------- DIAG layout ----------------
  if (P->structure == LORADS_STRUCT_DIAG) {
    std::vector<int> drow(m);
    std::vector<double> dcoef(m);
    for (int i = 0; i < m; ++i) {
      drow[i] = krow[kptr[i]];
      dcoef[i] = kval[kptr[i]];
    }
    std::vector<int> dptr;
    csr_counts(drow, n, dptr);
    std::vector<double> dsq(n, 0.0);
    for (int i = 0; i < m; ++i) dsq[drow[i]] += dcoef[i] * dcoef[i];
    P->drow.upload(drow, s);
    P->dptr.upload(dptr, s);
    P->dcoef.upload(dcoef, s);
    P->dsq.upload(dsq, s);
    std::vector<float> f1(dcoef.begin(), dcoef.end()), f2(dsq.begin(), dsq.end());
    P->dcoeff.upload(f1, s);
    P->dsqf.upload(f2, s);
  }
  // ---------------- PAIR layout ----------------
  if (P->structure == LORADS_STRUCT_PAIR) {
    std::vector<int> pj(m), pk(m);
    std::vector<double> pc(m);
    bool uniform = true;
    for (int i = 0; i < m; ++i) {
      pj[i] = krow[kptr[i]];
      pk[i] = kcol[kptr[i]];
      pc[i] = kval[kptr[i]];
      if (pc[i] != pc[0]) uniform = false;
    }
    std::vector<int> rptr;
    csr_counts(pj, n, rptr);
    // incident lists: constraint i joins the list of row pj[i] (partner pk[i])
    // and of row pk[i] (partner pj[i]).  Filling in internal order (sorted by
    // (j, k)) leaves every list sorted by partner: a row's entries as the
    // larger index (partners j < row) all precede its entries as the smaller.
    std::vector<int> inc_ptr(n + 1, 0);
    for (int i = 0; i < m; ++i) { ++inc_ptr[pj[i] + 1]; ++inc_ptr[pk[i] + 1]; }
    for (int j = 0; j < n; ++j) inc_ptr[j + 1] += inc_ptr[j];
    std::vector<int> inc_nb(2 * (size_t)m), inc_id(2 * (size_t)m);
    {
      std::vector<int> pos(inc_ptr.begin(), inc_ptr.end() - 1);
      for (int i = 0; i < m; ++i) {
        int t = pos[pj[i]]++;
        inc_nb[t] = pk[i];
        inc_id[t] = i;
        t = pos[pk[i]]++;
        inc_nb[t] = pj[i];
        inc_id[t] = i;
      }
    }
    P->pj.upload(pj, s);
    P->pk.upload(pk, s);
    if (uniform) {
      P->pair_coef = pc[0];
    } else {
      P->pcoef.upload(pc, s);
      std::vector<float> f(pc.begin(), pc.end());
      P->pcoeff.upload(f, s);
    }
    P->rptr.upload(rptr, s);
    {
      std::vector<int> crow, cstart;
      for (int j = 0; j < n; ++j)
        for (int i = rptr[j]; i < rptr[j + 1]; i += kPairChunk) {
          crow.push_back(j);
          cstart.push_back(i);
        }
      P->nfchunks = (int)crow.size();
      P->fchunk_row.upload(crow, s);
      P->fchunk_start.upload(cstart, s);
    }
    {
      // XCD chunk lists of the two-column FP64 maps: partner rows are cut into
      // kXcds blocks of about m / kXcds constraints each (quantiles of the
      // partner index); list x holds, row after row, the pieces of each row's
      // run (sorted by partner) whose partners lie in block x, cut into near
      // equal chunks of at most kPairChunk.  Workgroups b with b mod kXcds = x
      // serve list x, so an XCD gathers partner rows from one block only.
      std::vector<long long> cum(n + 1, 0);
      for (int i = 0; i < m; ++i) ++cum[pk[i] + 1];
      for (int k = 0; k < n; ++k) cum[k + 1] += cum[k];
      std::vector<int> kb(kXcds + 1, n);
      kb[0] = 0;
      for (int x = 1; x < kXcds; ++x) {
        const long long want = (long long)m * x / kXcds;
        kb[x] = (int)(std::lower_bound(cum.begin(), cum.end(), want) - cum.begin());
        kb[x] = std::max(kb[x], kb[x - 1]);
      }
      std::vector<int> xr[kXcds], xs[kXcds], xe[kXcds];
      for (int j = 0; j < n; ++j) {
        int i = rptr[j];
        for (int x = 0; x < kXcds; ++x) {
          int e = i;
          while (e < rptr[j + 1] && pk[e] < kb[x + 1]) ++e;
          const int len = e - i;
          if (len > 0) {
            const int pieces = (len + kPairChunk - 1) / kPairChunk;
            for (int q = 0; q < pieces; ++q) {
              xr[x].push_back(j);
              xs[x].push_back(i + (int)((long long)len * q / pieces));
              xe[x].push_back(i + (int)((long long)len * (q + 1) / pieces));
            }
          }
          i = e;
        }
      }
      std::vector<int> row, start, end, off(kXcds + 1, 0);
      int maxlen = 0;
      for (int x = 0; x < kXcds; ++x) {
        off[x + 1] = off[x] + (int)xr[x].size();
        maxlen = std::max(maxlen, (int)xr[x].size());
        row.insert(row.end(), xr[x].begin(), xr[x].end());
        start.insert(start.end(), xs[x].begin(), xs[x].end());
        end.insert(end.end(), xe[x].begin(), xe[x].end());
      }
      P->xchunk_row.upload(row, s);
      P->xchunk_start.upload(start, s);
      P->xchunk_end.upload(end, s);
      P->xchunk_off.upload(off, s);
      P->nxchunks = (int)row.size();
      P->xchunk_maxlen = maxlen;
    }
    P->inc_ptr.upload(inc_ptr, s);
    P->inc_nb.upload(inc_nb, s);
    P->inc_id.upload(inc_id, s);
    {
      // partner blocks of the incident entries (2m / kXcds each) and every
      // row's runs per block (its list is sorted by partner)
      std::vector<long long> cum(n + 1, 0);
      for (size_t t = 0; t < inc_nb.size(); ++t) ++cum[inc_nb[t] + 1];
      for (int k = 0; k < n; ++k) cum[k + 1] += cum[k];
      std::vector<int> kb(kXcds + 1, n);
      kb[0] = 0;
      for (int x = 1; x < kXcds; ++x) {
        const long long want = 2LL * m * x / kXcds;
        kb[x] = std::max(kb[x - 1], (int)(std::lower_bound(cum.begin(), cum.end(), want) - cum.begin()));
      }
      std::vector<int> xp((size_t)n * (kXcds + 1));
      for (int t = 0; t < n; ++t) {
        int e = inc_ptr[t];
        for (int x = 0; x < kXcds; ++x) {
          xp[(size_t)t * (kXcds + 1) + x] = e;
          while (e < inc_ptr[t + 1] && inc_nb[e] < kb[x + 1]) ++e;
        }
        xp[(size_t)t * (kXcds + 1) + kXcds] = inc_ptr[t + 1];
      }
      P->inc_xptr.upload(xp, s);
    }
    if (uniform) {
      std::vector<double> lb(2 * inc_id.size(), 0.0);
      for (size_t t = 0; t < inc_id.size(); ++t) lb[2 * t + 1] = b_int[inc_id[t]];
      P->inc_lb.upload(lb, s);
    }
    bool upper_view = true;
    for (int j = 0; j < n && upper_view; ++j) {
      const int nup = rptr[j + 1] - rptr[j];
      const int lo = inc_ptr[j + 1] - nup;
      if (lo < inc_ptr[j]) { upper_view = false; break; }
      for (int q = 0; q < nup; ++q)
        if (inc_id[lo + q] != rptr[j] + q) { upper_view = false; break; }
    }
    P->inc_upper_view = upper_view;
  }

  P->kptr.upload(kptr, s);
  P->krow.upload(krow, s);
  P->kcol.upload(kcol, s);
  P->kval.upload(kval, s);
  {
    std::vector<float> kf(kval.begin(), kval.end());
    P->kvalf.upload(kf, s);
  }
  P->b.upload(b_int, s);
  if (!P->perm_identity) P->perm.upload(perm, s);

  P->sc.alloc(S_COUNT);
  P->sc.zero(s);
  // one partial per block of the widest row kernel (64 lanes per row)
  // (the PAIR adjoint runs one block per row)
  P->part_cap = std::max<size_t>(kMaxPart, (size_t)n + 64);
  P->part.alloc(P->part_cap);
  P->zbuf.alloc(m);
  P->wbuf.alloc(m);
  P->tbuf.alloc(m);
  P->tbuff.alloc(m);
  HIPCHK(hipStreamSynchronize(s));
  return P;
}

}  // namespace lorads
