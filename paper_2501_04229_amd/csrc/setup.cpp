// Host side of gadi_setup: CSR validation, the Hermitian/skew-Hermitian
// splitting H = (A + A^T)/2, S = (A - A^T)/2 (Section 4.1 of the paper) on the
// union pattern of A and A^T, and packing into the SELL-64 device layout.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <vector>

#include "internal.h"

namespace gadi {

gadi_status fail_hip(hipError_t e, const char* what, const char* file, int line) {
  if (std::getenv("GADI_DEBUG"))
    std::fprintf(stderr, "gadi: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
  return e == hipErrorOutOfMemory ? GADI_ENOMEM : GADI_EHIP;
}

// IEEE binary64 -> binary16 with one round-to-nearest-even step (no detour
// through binary32, which could round twice).
static uint16_t f64_to_f16_rne(double d) {
  uint64_t u;
  std::memcpy(&u, &d, sizeof u);
  uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
  int bexp = (int)((u >> 52) & 0x7ff);
  uint64_t mant = u & ((1ull << 52) - 1);
  if (bexp == 0x7ff) return (uint16_t)(sign | 0x7c00u | (mant ? 0x200u : 0u));
  if (bexp == 0) return sign;  // binary64 subnormals are far below binary16's range
  int e = bexp - 1023;
  if (e > 15) return (uint16_t)(sign | 0x7c00u);
  uint64_t m = mant | (1ull << 52);
  int shift;
  uint32_t hexp;
  if (e >= -14) {
    shift = 42;
    hexp = (uint32_t)(e + 15);
  } else {
    shift = 42 + (-14 - e);
    hexp = 0;
  }
  if (shift >= 64) return sign;
  uint64_t q = m >> shift;
  uint64_t rem = m & ((1ull << shift) - 1);
  uint64_t halfway = 1ull << (shift - 1);
  if (rem > halfway || (rem == halfway && (q & 1))) ++q;
  if (hexp == 0) return (uint16_t)(sign | (uint16_t)q);  // q == 1024 encodes the smallest normal
  if (q == 2048) {
    q = 1024;
    ++hexp;
  }
  if (hexp >= 31) return (uint16_t)(sign | 0x7c00u);
  return (uint16_t)(sign | (hexp << 10) | (uint32_t)(q - 1024));
}

template <class T>
static gadi_status upload(T** dst, const std::vector<T>& src) {
  size_t bytes = src.size() * sizeof(T);
  GADI_HIP_CHECK(hipMalloc((void**)dst, bytes ? bytes : sizeof(T)));
  if (bytes) GADI_HIP_CHECK(hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice));
  return GADI_OK;
}

gadi_status ensure_fp8_public(System& s);

void free_system(System& s) {
  void* ptrs[] = {s.slice_dia, s.dia_off, s.slice_ptr, s.col,     s.a_off,   s.a_diag,  s.h_off64, s.s_off64, s.h_diag64,
                  s.h_off16,   s.s_off16, s.h_diag16, s.h_off32, s.s_off32, s.h_diag32, s.a_off32, s.a_diag32, s.ws,
                  s.hist,      s.sync,    s.flags,   s.part,    s.result,  s.info, s.prof, s.h_off8, s.s_off8};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < 4; ++k) {
    if (s.h_half[k]) (void)hipFree(s.h_half[k]);
    if (s.s_half[k]) (void)hipFree(s.s_half[k]);
  }
  if (s.ev0) (void)hipEventDestroy(s.ev0);
  if (s.ev1) (void)hipEventDestroy(s.ev1);
  s = System();
}

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_setup(const gadi_csr* A, gadi_splitting split, gadi_handle** out) {
  if (!out) return GADI_EINVAL;
  *out = nullptr;
  if (!A || split != GADI_SPLIT_HSS) return GADI_EINVAL;
  const int n = A->n;
  const int64_t nnz = A->nnz;
  // n <= kMaxRows: every solver vector of doubles stays below 4 GiB (32-bit byte offsets)
  if (n < 1 || n > kMaxRows || nnz < 0 || nnz >= (int64_t(1) << 31) || !A->row_ptr ||
      (nnz > 0 && (!A->col_idx || !A->val)))
    return GADI_EINVAL;

  std::vector<int32_t> rp(n + 1), col;
  std::vector<double> val;
  try {
    col.resize(nnz);
    val.resize(nnz);
  } catch (const std::bad_alloc&) {
    return GADI_ENOMEM;
  }
  if (A->on_device) {
    GADI_HIP_CHECK(hipMemcpy(rp.data(), A->row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (nnz) {
      GADI_HIP_CHECK(hipMemcpy(col.data(), A->col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      GADI_HIP_CHECK(hipMemcpy(val.data(), A->val, nnz * sizeof(double), hipMemcpyDeviceToHost));
    }
  } else {
    std::memcpy(rp.data(), A->row_ptr, (n + 1) * sizeof(int32_t));
    if (nnz) {
      std::memcpy(col.data(), A->col_idx, nnz * sizeof(int32_t));
      std::memcpy(val.data(), A->val, nnz * sizeof(double));
    }
  }
  // validation: monotone row pointers, in-range strictly increasing columns
  if (rp[0] != 0 || rp[n] != nnz) return GADI_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return GADI_EINVAL;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) return GADI_EINVAL;
      if (k > rp[i] && col[k] <= col[k - 1]) return GADI_EINVAL;
    }
  }

  // A^T by counting sort (columns of each transposed row come out ascending)
  std::vector<int32_t> trp(n + 1, 0), tcol;
  std::vector<double> tval;
  try {
    tcol.resize(nnz);
    tval.resize(nnz);
  } catch (const std::bad_alloc&) {
    return GADI_ENOMEM;
  }
  for (int64_t k = 0; k < nnz; ++k) trp[col[k] + 1]++;
  for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
  {
    std::vector<int32_t> next(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        int d = next[col[k]]++;
        tcol[d] = i;
        tval[d] = val[k];
      }
  }

  // Walk row i of A and of A^T together: calls f(col, a_ij, a_ji) per column
  // of the union pattern in ascending order.
  auto merge_row = [&](int i, auto&& f) {
    int ka = rp[i], ea = rp[i + 1], kt = trp[i], et = trp[i + 1];
    while (ka < ea || kt < et) {
      int ca = ka < ea ? col[ka] : n;
      int ct = kt < et ? tcol[kt] : n;
      int c = ca < ct ? ca : ct;
      double va = 0.0, vt = 0.0;
      if (ca == c) va = val[ka++];
      if (ct == c) vt = tval[kt++];
      f(c, va, vt);
    }
  };

  const int npad = (n + kPadRows - 1) / kPadRows * kPadRows;
  const int nslices = npad / kSlice;
  // Per slice: the longest row (SELL width) and the distinct column offsets
  // col - row of its off-diagonal entries.  A slice with at most kDiaMax
  // distinct offsets is stored diagonal-style: one slot per offset (ascending),
  // zero-valued phantom entries where a row lacks that offset, no per-entry
  // column index.  Every slice of a stencil matrix qualifies.
  std::vector<int32_t> width(nslices, 0), is_dia(nslices, 1), nofs(nslices, 0);
  std::vector<int32_t> dia_off((size_t)nslices * kDiaMax, 0);
  int64_t nnz_off = 0;
  for (int i = 0; i < n; ++i) {
    const int s = i / kSlice;
    int cnt = 0;
    int32_t* offs = &dia_off[(size_t)s * kDiaMax];
    merge_row(i, [&](int c, double, double) {
      if (c == i) return;
      ++cnt;
      if (!is_dia[s]) return;
      const int32_t d = c - i;
      int k = 0;
      while (k < nofs[s] && offs[k] != d) ++k;
      if (k == nofs[s]) {
        if (nofs[s] == kDiaMax) is_dia[s] = 0;
        else offs[nofs[s]++] = d;
      }
    });
    nnz_off += cnt;
    if (cnt > width[s]) width[s] = cnt;
  }
  int64_t dia_slices = 0;
  for (int s = 0; s < nslices; ++s) {
    if (is_dia[s]) {
      std::sort(dia_off.begin() + (size_t)s * kDiaMax, dia_off.begin() + (size_t)s * kDiaMax + nofs[s]);
      width[s] = nofs[s];
      ++dia_slices;
    } else {
      nofs[s] = 0;
    }
  }
  // Uniform diagonal-style layout: if every slice is diagonal-style and the
  // union of their offsets has 4 or 6 members (the 2-D and 3-D stencils), every
  // slice is stored with the union's offsets, phantom zeros where a slice
  // lacks one, as long as that adds at most a quarter to the stored slots of
  // the slices that hold rows.
  // The solver then takes the offsets from its arguments instead of reading
  // per-slice metadata.
  int dia_uniform = 0;
  std::vector<int32_t> uni;
  if (dia_slices == nslices) {
    int64_t slots_before = 0;
    for (int s = 0; s < nslices; ++s) {
      slots_before += (int64_t)width[s] * kSlice;
      for (int k = 0; k < nofs[s]; ++k) uni.push_back(dia_off[(size_t)s * kDiaMax + k]);
      if (uni.size() > 64) {  // keep the candidate set small while scanning
        std::sort(uni.begin(), uni.end());
        uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
        if (uni.size() > (size_t)kDiaMax) break;
      }
    }
    std::sort(uni.begin(), uni.end());
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    // trailing slices past row n - 1 (tile padding) hold no rows: not counted
    const int64_t used_slices = (n + kSlice - 1) / kSlice;
    const int64_t slots_after = (int64_t)uni.size() * used_slices * kSlice;
    // (double values of the uniform layout are addressed with 32-bit byte offsets)
    if ((uni.size() == 4 || uni.size() == 6) && slots_after <= slots_before + slots_before / 4 &&
        (int64_t)uni.size() * npad * (int64_t)sizeof(double) < (int64_t(1) << 32)) {
      dia_uniform = (int)uni.size();
      for (int s = 0; s < nslices; ++s) {
        nofs[s] = dia_uniform;
        width[s] = dia_uniform;
        for (int k = 0; k < dia_uniform; ++k) dia_off[(size_t)s * kDiaMax + k] = uni[k];
      }
    }
  }
  std::vector<int32_t> slice_ptr(nslices + 1, 0);
  int64_t acc = 0;
  int max_width = 0;
  for (int s = 0; s < nslices; ++s) {
    slice_ptr[s] = (int32_t)acc;
    acc += (int64_t)width[s] * kSlice;
    if (acc >= (int64_t(1) << 31)) return GADI_EINVAL;
    if (width[s] > max_width) max_width = width[s];
  }
  slice_ptr[nslices] = (int32_t)acc;
  const int64_t nslots = acc;

  std::vector<int32_t> hcol;
  std::vector<double> a_off, h64, s64, a_diag(npad, 0.0), h_diag64(npad, 0.0);
  std::vector<uint16_t> h16, s16, hd16(npad, 0);
  try {
    hcol.resize(nslots);
    a_off.assign(nslots, 0.0);
    h64.assign(nslots, 0.0);
    s64.assign(nslots, 0.0);
    h16.assign(nslots, 0);
    s16.assign(nslots, 0);
  } catch (const std::bad_alloc&) {
    return GADI_ENOMEM;
  }
  // Empty slots: in explicit slices they point at their own row (rows past n
  // at row n - 1, so a product with a caller's length-n vector never reads
  // past its end); in diagonal-style slices the kernels never read the column
  // array, which marks phantom entries with -1.
  for (int s = 0; s < nslices; ++s)
    for (int j = 0; j < width[s]; ++j)
      for (int l = 0; l < kSlice; ++l) {
        const int row = s * kSlice + l;
        hcol[slice_ptr[s] + (int64_t)j * kSlice + l] = is_dia[s] ? -1 : (row < n ? row : n - 1);
      }
  for (int i = 0; i < n; ++i) {
    const int s = i / kSlice, l = i % kSlice;
    const int32_t* offs = &dia_off[(size_t)s * kDiaMax];
    int j = 0;
    merge_row(i, [&](int c, double va, double vt) {
      double hv = (va + vt) / 2.0, sv = (va - vt) / 2.0;
      if (c == i) {
        a_diag[i] = va;
        h_diag64[i] = hv;
        hd16[i] = f64_to_f16_rne(hv);
        return;
      }
      int slot = j++;
      if (is_dia[s]) {
        slot = 0;
        while (offs[slot] != c - i) ++slot;
      }
      int64_t k = slice_ptr[s] + (int64_t)slot * kSlice + l;
      hcol[k] = c;
      a_off[k] = va;
      h64[k] = hv;
      s64[k] = sv;
      h16[k] = f64_to_f16_rne(hv);
      s16[k] = f64_to_f16_rne(sv);
    });
  }
  // free the host CSR copies before allocating device memory
  std::vector<int32_t>().swap(col);
  std::vector<double>().swap(val);
  std::vector<int32_t>().swap(tcol);
  std::vector<double>().swap(tval);

  gadi_handle* h = new (std::nothrow) gadi_handle();
  if (!h) return GADI_ENOMEM;
  System& S = h->sys;
  S.n = n;
  S.npad = npad;
  S.nslices = nslices;
  S.nnz_a = nnz;
  S.nnz_off = nnz_off;
  S.nslots = nslots;
  S.max_width = max_width;
  S.dia_slices = dia_slices;
  S.dia_uniform = dia_uniform;
  for (int k = 0; k < dia_uniform; ++k) S.dia_u[k] = uni[k];
  S.dia_sym = dia_uniform > 0;
  for (int k = 0; k < dia_uniform; ++k)
    if (uni[k] != -uni[dia_uniform - 1 - k]) S.dia_sym = false;
  int64_t dslots = 0, expl = 0;
  for (int sl = 0; sl < nslices; ++sl) {
    const int64_t slots = (int64_t)(slice_ptr[sl + 1] - slice_ptr[sl]);
    if (is_dia[sl]) dslots += slots;
  }
  for (int sl = 0; sl < nslices; ++sl) {
    if (is_dia[sl]) continue;
    for (int64_t k = slice_ptr[sl]; k < slice_ptr[sl + 1]; ++k) {
      const int row = sl * kSlice + (int)((k - slice_ptr[sl]) % kSlice);
      if (row < n && hcol[k] != row) ++expl;
    }
  }
  S.dia_slots = dslots;
  S.explicit_entries = expl;
  (void)hipGetDevice(&S.device);
  gadi_status st = GADI_OK;
  if ((st = upload(&S.slice_ptr, slice_ptr)) != GADI_OK || (st = upload(&S.col, hcol)) != GADI_OK ||
      (st = upload(&S.a_off, a_off)) != GADI_OK || (st = upload(&S.a_diag, a_diag)) != GADI_OK ||
      (st = upload(&S.h_off64, h64)) != GADI_OK || (st = upload(&S.s_off64, s64)) != GADI_OK ||
      (st = upload(&S.h_diag64, h_diag64)) != GADI_OK || (st = upload(&S.slice_dia, nofs)) != GADI_OK ||
      (st = upload(&S.dia_off, dia_off)) != GADI_OK ||
      (st = upload((uint16_t**)&S.h_off16, h16)) != GADI_OK ||
      (st = upload((uint16_t**)&S.s_off16, s16)) != GADI_OK ||
      (st = upload((uint16_t**)&S.h_diag16, hd16)) != GADI_OK) {
    free_system(S);
    delete h;
    return st;
  }
  *out = h;
  return GADI_OK;
}

extern "C" gadi_status gadi_destroy(gadi_handle* h) {
  if (!h) return GADI_EINVAL;
  free_system(h->sys);
  delete h;
  return GADI_OK;
}

extern "C" gadi_status gadi_set_stream(gadi_handle* h, void* stream) {
  if (!h) return GADI_EINVAL;
  h->sys.stream = (hipStream_t)stream;
  return GADI_OK;
}

extern "C" const char* gadi_status_str(gadi_status s) {
  switch (s) {
    case GADI_OK: return "ok";
    case GADI_EINVAL: return "invalid argument";
    case GADI_ENOTSPD: return "inner operator not positive definite";
    case GADI_EOVERFLOW16: return "half-precision overflow";
    case GADI_EDIVERGED: return "diverged";
    case GADI_EMAXIT: return "outer sweep limit reached";
    case GADI_EHIP: return "HIP runtime error";
    case GADI_ENOMEM: return "out of memory";
    case GADI_EBARRIER: return "device barrier timed out";
    case GADI_EPRUNED: return "pruned: dominated by a converged trial";
  }
  return "unknown status";
}

extern "C" void gadi_default_options(gadi_options* o, gadi_precision prec) {
  if (!o) return;
  o->prec = prec;
  // inexact inner solves: the refinement corrects what they leave, and at 3e-2
  // the sweep count barely grows while the inner steps drop by a third
  o->eps_inner = prec == GADI_PREC_FP64 ? 1e-6 : 3e-2;
  o->maxit_outer = 20000;
  o->maxit_inner = 2000;
  o->on_device = 0;
  o->record_history = 0;
  o->prune_dominated = 0;
  o->grid_per_system = 0;
}

extern "C" gadi_status gadi_get_layout(gadi_handle* h, int64_t* out) {
  if (!h || !out) return GADI_EINVAL;
  const System& S = h->sys;
  out[0] = S.n;
  out[1] = S.npad;
  out[2] = S.nnz_off;
  out[3] = S.nslots;
  out[4] = S.dia_slots;
  out[5] = S.explicit_entries;
  out[6] = S.dia_uniform;
  return GADI_OK;
}

extern "C" gadi_status gadi_get_split_fp16(gadi_handle* h, int32_t which, int32_t* out_rp, int32_t* out_col,
                                           uint16_t* out_val, int64_t* nnz_out) {
  if (!h || (which != 1 && which != 2)) return GADI_EINVAL;
  System& S = h->sys;
  const int64_t total = S.nnz_off + S.n;  // off-diagonals plus one diagonal per row
  if (nnz_out) *nnz_out = total;
  if (!out_rp && !out_col && !out_val) return GADI_OK;
  if (!out_rp || !out_col || !out_val) return GADI_EINVAL;
  std::vector<int32_t> sp(S.nslices + 1), c(S.nslots);
  std::vector<uint16_t> v(S.nslots), d(S.npad);
  GADI_HIP_CHECK(hipMemcpy(sp.data(), S.slice_ptr, sp.size() * 4, hipMemcpyDeviceToHost));
  GADI_HIP_CHECK(hipMemcpy(c.data(), S.col, c.size() * 4, hipMemcpyDeviceToHost));
  GADI_HIP_CHECK(hipMemcpy(v.data(), which == 1 ? (void*)S.h_off16 : (void*)S.s_off16, v.size() * 2,
                           hipMemcpyDeviceToHost));
  GADI_HIP_CHECK(hipMemcpy(d.data(), S.h_diag16, d.size() * 2, hipMemcpyDeviceToHost));
  int64_t pos = 0;
  out_rp[0] = 0;
  for (int i = 0; i < S.n; ++i) {
    int s = i / kSlice, l = i % kSlice;
    int w = (sp[s + 1] - sp[s]) / kSlice;
    bool diag_done = false;
    for (int j = 0; j <= w; ++j) {
      int cj = -1;
      uint16_t vj = 0;
      if (j < w) {
        int64_t k = sp[s] + (int64_t)j * kSlice + l;
        if (c[k] == i || c[k] < 0) continue;  // padding or phantom
        cj = c[k];
        vj = v[k];
      }
      if (!diag_done && (j == w || cj > i)) {
        out_col[pos] = i;
        out_val[pos] = which == 1 ? d[i] : (uint16_t)0;
        ++pos;
        diag_done = true;
      }
      if (j < w) {
        out_col[pos] = cj;
        out_val[pos] = vj;
        ++pos;
      }
    }
    out_rp[i + 1] = (int32_t)pos;
  }
  return GADI_OK;
}

extern "C" gadi_status gadi_get_split_fp8(gadi_handle* h, int32_t which, int32_t* out_rp, int32_t* out_col,
                                          uint8_t* out_val, int64_t* nnz_out) {
  if (!h || (which != 1 && which != 2)) return GADI_EINVAL;
  System& S = h->sys;
  if (nnz_out) *nnz_out = S.nnz_off;
  if (!out_rp && !out_col && !out_val) return GADI_OK;
  if (!out_rp || !out_col || !out_val) return GADI_EINVAL;
  GADI_HIP_CHECK(hipSetDevice(S.device));
  const gadi_status st = ensure_fp8_public(S);
  if (st != GADI_OK) return st;
  std::vector<int32_t> sp(S.nslices + 1), c(S.nslots);
  std::vector<uint8_t> v(S.nslots);
  GADI_HIP_CHECK(hipMemcpy(sp.data(), S.slice_ptr, sp.size() * 4, hipMemcpyDeviceToHost));
  GADI_HIP_CHECK(hipMemcpy(c.data(), S.col, c.size() * 4, hipMemcpyDeviceToHost));
  GADI_HIP_CHECK(hipMemcpy(v.data(), which == 1 ? S.h_off8 : S.s_off8, v.size(), hipMemcpyDeviceToHost));
  // slots of a row hold its off-diagonal entries in ascending column order
  int64_t pos = 0;
  out_rp[0] = 0;
  for (int i = 0; i < S.n; ++i) {
    const int s = i / kSlice, l = i % kSlice;
    const int w = (sp[s + 1] - sp[s]) / kSlice;
    for (int j = 0; j < w; ++j) {
      const int64_t k = sp[s] + (int64_t)j * kSlice + l;
      if (c[k] == i || c[k] < 0) continue;  // padding or phantom
      out_col[pos] = c[k];
      out_val[pos] = v[k];
      ++pos;
    }
    out_rp[i + 1] = (int32_t)pos;
  }
  return GADI_OK;
}
