// Host-only parts of the C ABI: the direct-product-decomposition layout, the
// algorithmic flop count and the status strings.
//
// Layout (paper, symmetry section): a tensor element is stored only when the
// product (XOR) of its index irreps is the totally symmetric irrep; pair
// indices of a doubles tensor are grouped by pair irrep G.
#include <cstring>

#include "../../include/cdcc.h"

namespace {

bool valid_h(int h) { return h == 1 || h == 2 || h == 4 || h == 8; }

// Number of pairs x>=y (orbital order: irrep, then local index) of pair irrep
// G from per-irrep counts n[].
int64_t packed_pairs(const int32_t *n, int h, int G) {
  int64_t s = 0;
  for (int g = 0; g < h; ++g) {
    const int g2 = g ^ G;
    if (g > g2) s += int64_t(n[g]) * n[g2];
    else if (g == g2) s += int64_t(n[g]) * (n[g] + 1) / 2;
  }
  return s;
}

// Strict version (x>y).
int64_t strict_pairs(const int32_t *n, int h, int G) {
  int64_t s = 0;
  for (int g = 0; g < h; ++g) {
    const int g2 = g ^ G;
    if (g > g2) s += int64_t(n[g]) * n[g2];
    else if (g == g2) s += int64_t(n[g]) * (n[g] - 1) / 2;
  }
  return s;
}

}  // namespace

extern "C" int cdcc_irrep_layout(const cdcc_sym_t *sym, cdcc_layout_t *out) {
  if (!sym || !out) return CDCC_EINVAL;
  const int h = sym->nirrep;
  if (!valid_h(h)) return CDCC_EUNSUPPORTED;
  for (int g = 0; g < h; ++g)
    if (sym->nocc[g] < 0 || sym->nvir[g] < 0 || sym->ncd[g] < 0) return CDCC_EINVAL;
  cdcc_layout_t L;
  std::memset(&L, 0, sizeof(L));
  L.sym = *sym;
  for (int g = h; g < CDCC_MAX_IRREP; ++g) L.sym.nocc[g] = L.sym.nvir[g] = L.sym.ncd[g] = 0;
  const int32_t *no = L.sym.nocc, *nv = L.sym.nvir, *nc = L.sym.ncd;
  int64_t amp = 0;
  for (int G = 0; G < h; ++G) {
    int64_t ro = 0, rv = 0;
    for (int g = 0; g < h; ++g) {
      L.oo_off[G][g] = ro;
      L.vv_off[G][g] = rv;
      ro += int64_t(no[g]) * no[g ^ G];
      rv += int64_t(nv[g]) * nv[g ^ G];
    }
    L.n_oo[G] = ro;
    L.n_vv[G] = rv;
    L.n_oo_pk[G] = packed_pairs(no, h, G);
    L.n_vv_pk[G] = packed_pairs(nv, h, G);
    L.amp_off[G] = amp;
    amp += ro * rv;
  }
  L.amp_size = amp;
  int64_t ob = 0, ov = 0;
  for (int gP = 0; gP < h; ++gP)
    for (int ga = 0; ga < h; ++ga) {
      L.b_off[gP][ga] = ob;
      L.bvo_off[gP][ga] = ov;
      ob += int64_t(nv[ga]) * nv[ga ^ gP] * nc[gP];
      ov += int64_t(nv[ga]) * no[ga ^ gP] * nc[gP];
    }
  L.b_size = ob;
  L.bvo_size = ov;
  int64_t ot = 0, oo = 0, vo = 0, co = 0;
  for (int g = 0; g < h; ++g) {
    L.t1_off[g] = ot;
    L.occ_off[g] = oo;
    L.vir_off[g] = vo;
    L.cd_off[g] = co;
    ot += int64_t(no[g]) * nv[g];
    oo += no[g];
    vo += nv[g];
    co += nc[g];
  }
  L.t1_size = ot;
  L.nocc_tot = oo;
  L.nvir_tot = vo;
  L.ncd_tot = co;
  *out = L;
  return CDCC_OK;
}

// F_W = sum_{Ga>=Gb} npk(Ga,Gb) sum_GP 2 kappa N_GP v_{Ga^GP} v_{Gb^GP}
// F_C = sum_{Ga>=Gb} sum_{Gc>=Gd, Gc^Gd=Ga^Gb, W!=0} 2 [n+oo n+ab n+cd + n-oo n-ab n-cd]
// F_dress = sum_GP sum_Ga 2 o_{Ge} v_{Ge} v_{Ga} N_GP   (Ge = Ga^GP)
extern "C" int cdcc_ladder_flops(const cdcc_layout_t *lay, int32_t kind, double flops[3]) {
  if (!lay || !flops || kind < 0 || kind > 2) return CDCC_EINVAL;
  const int h = lay->sym.nirrep;
  if (!valid_h(h)) return CDCC_EUNSUPPORTED;
  const int32_t *no = lay->sym.nocc, *nv = lay->sym.nvir, *nc = lay->sym.ncd;
  const double kappa = kind == 0 ? 1.0 : 2.0;
  auto npair = [&](int g1, int g2, bool strict) -> double {
    if (g1 > g2) return double(nv[g1]) * nv[g2];
    if (g1 == g2) return strict ? double(nv[g1]) * (nv[g1] - 1) / 2 : double(nv[g1]) * (nv[g1] + 1) / 2;
    return 0.0;
  };
  double fw = 0, fc = 0, fd = 0;
  for (int ga = 0; ga < h; ++ga)
    for (int gb = 0; gb <= ga; ++gb) {
      const int G = ga ^ gb;
      double w = 0;
      for (int gP = 0; gP < h; ++gP) w += 2.0 * kappa * nc[gP] * double(nv[ga ^ gP]) * nv[gb ^ gP];
      fw += npair(ga, gb, false) * w;
      const double noo_p = double(packed_pairs(no, h, G)), noo_m = double(strict_pairs(no, h, G));
      for (int gc = 0; gc < h; ++gc) {
        const int gd = gc ^ G;
        if (gc < gd) continue;
        if (nc[ga ^ gc] == 0 && nc[ga ^ gd] == 0) continue;  // W block is zero
        fc += 2.0 * (noo_p * npair(ga, gb, false) * npair(gc, gd, false) +
                     noo_m * npair(ga, gb, true) * npair(gc, gd, true));
      }
    }
  if (kind == 2)
    for (int gP = 0; gP < h; ++gP)
      for (int ga = 0; ga < h; ++ga) {
        const int ge = ga ^ gP;
        fd += 2.0 * no[ge] * double(nv[ge]) * nv[ga] * nc[gP];
      }
  flops[0] = fw;
  flops[1] = fc;
  flops[2] = fd;
  return CDCC_OK;
}

extern "C" int cdcc_density_flops(const cdcc_layout_t *lay, double flops[2]) {
  if (!lay || !flops) return CDCC_EINVAL;
  const int h = lay->sym.nirrep;
  if (!valid_h(h)) return CDCC_EUNSUPPORTED;
  const int32_t *no = lay->sym.nocc, *nv = lay->sym.nvir, *nc = lay->sym.ncd;
  auto n_oo = [&](int G) {
    double n = 0;
    for (int g = 0; g < h; ++g) n += double(no[g]) * no[g ^ G];
    return n;
  };
  auto n_vv = [&](int G) {
    double n = 0;
    for (int g = 0; g < h; ++g) n += double(nv[g]) * nv[g ^ G];
    return n;
  };
  double fv = 0, fl = 0;
  for (int gP = 0; gP < h; ++gP) {
    if (nc[gP] == 0) continue;
    for (int ga = 0; ga < h; ++ga) {
      const int gc = ga ^ gP;
      for (int gb = 0; gb < h; ++gb) {
        const int gd = gb ^ gP;
        fv += 4.0 * double(nv[ga]) * nv[gb] * nv[gc] * nv[gd] * n_oo(ga ^ gb);
      }
      fl += 2.0 * double(nv[ga]) * nv[gc] * n_vv(gP) * nc[gP];
    }
  }
  flops[0] = fv;
  flops[1] = fl;
  return CDCC_OK;
}

extern "C" int cdcc_vo_layout(const cdcc_layout_t *lay, cdcc_vo_layout_t *out) {
  if (!lay || !out) return CDCC_EINVAL;
  const int h = lay->sym.nirrep;
  if (!valid_h(h)) return CDCC_EUNSUPPORTED;
  const int32_t *no = lay->sym.nocc, *nv = lay->sym.nvir;
  *out = cdcc_vo_layout_t{};
  int64_t ol = 0, om = 0;
  for (int G = 0; G < h; ++G) {
    int64_t r = 0;
    for (int gb = 0; gb < h; ++gb) {
      out->vo_off[G][gb] = r;
      r += int64_t(nv[gb]) * no[gb ^ G];
    }
    out->n_vo[G] = r;
    out->lam_off[G] = ol;
    out->m_off[G] = om;
    ol += r * lay->n_oo[G];
    om += r * lay->n_vv[G];
  }
  out->lam_size = ol;
  out->m_size = om;
  return CDCC_OK;
}

extern "C" int cdcc_partial_flops(const cdcc_layout_t *lay, double flops[2]) {
  if (!lay || !flops) return CDCC_EINVAL;
  const int h = lay->sym.nirrep;
  if (!valid_h(h)) return CDCC_EUNSUPPORTED;
  const int32_t *no = lay->sym.nocc, *nv = lay->sym.nvir;
  double fs = 0, fa = 0;
  for (int G = 0; G < h; ++G) {
    double nvo = 0, kp = 0, km = 0, cp = 0, cm = 0;
    for (int g = 0; g < h; ++g) {
      nvo += double(nv[g]) * no[g ^ G];
      const int g2 = g ^ G;
      if (g > g2) {
        kp += double(no[g]) * no[g2];
        km += double(no[g]) * no[g2];
        cp += double(nv[g]) * nv[g2];
        cm += double(nv[g]) * nv[g2];
      } else if (g == g2) {
        kp += double(no[g]) * (no[g] + 1) / 2;
        km += double(no[g]) * (no[g] - 1) / 2;
        cp += double(nv[g]) * (nv[g] + 1) / 2;
        cm += double(nv[g]) * (nv[g] - 1) / 2;
      }
    }
    fs += 2.0 * nvo * kp * cp;
    fa += 2.0 * nvo * km * cm;
  }
  flops[0] = fs;
  flops[1] = fa;
  return CDCC_OK;
}

extern "C" const char *cdcc_status_string(int status) {
  switch (status) {
    case CDCC_OK: return "ok";
    case CDCC_EINVAL: return "invalid argument (layout, pointer, size or option)";
    case CDCC_ENOMEM: return "device workspace allocation failed";
    case CDCC_EUNSUPPORTED: return "unsupported (irrep count must be 1, 2, 4 or 8)";
    case CDCC_EDEVICE: return "HIP runtime error or no gfx950 device";
    case CDCC_ESCRATCH: return "problem needs more device memory than the static scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}
