// Launch side of the BF16 / FP16 partial-MTTKRP kernels (pm16_body.hpp; the
// kernels themselves are instantiated per storage type in pm16_bf16.hip and
// pm16_f16.hip): the pack of the first contracted factor into hi + lo values,
// then the partial MTTKRP, launched or recorded for the batched executor.
#include "pm_common.hpp"

namespace nncpk {

extern template const void* pm16_kernel_form<NNCP_BF16, false>(int, int, int, int, bool);
extern template const void* pm16_kernel_form<NNCP_BF16, true>(int, int, int, int, bool);
extern template const void* pm16_kernel_form<NNCP_F16, false>(int, int, int, int, bool);
extern template const void* pm16_kernel_form<NNCP_F16, true>(int, int, int, int, bool);
extern template const void* pm16_pack_kernel<NNCP_BF16>(bool);
extern template const void* pm16_pack_kernel<NNCP_F16>(bool);

namespace {

constexpr int left_tr16(int nb) { return nb >= 4 ? 4 : 8; }
constexpr int right_mc16(int nb) { return 4; }
constexpr int right_mc16_j1(int nb) { return nb >= 4 ? 9 : 8; }

const void* kernel16(int dtype, int side, int nb, int j1, int fast, int mt, bool batch) {
  if (dtype == NNCP_BF16)
    return mt ? pm16_kernel_form<NNCP_BF16, true>(side, nb, j1, fast, batch)
              : pm16_kernel_form<NNCP_BF16, false>(side, nb, j1, fast, batch);
  return mt ? pm16_kernel_form<NNCP_F16, true>(side, nb, j1, fast, batch)
            : pm16_kernel_form<NNCP_F16, false>(side, nb, j1, fast, batch);
}

void allow_big_lds(const void* k) { pm_allow_lds(k, 160 * 1024); }

}  // namespace

int pm_16_wave_rows(int side, int nb, int j1) {
  return side == 0 ? 16 * left_tr16(nb) : 16 * (j1 ? right_mc16_j1(nb) : right_mc16(nb));
}
int pm_16_kstep(int side) { return side == 0 ? 32 : 64; }
bool pm16_fast(int side, int64_t IL, int I1, int nb) {
  if (I1 % pm_16_kstep(side) != 0) return false;
  return side == 1 || IL % left_tr16(nb) == 0;
}
size_t pm_16_reduce_lds(int side, int nb, int wm) {
  if (wm >= 4) return 0;  // (also every J == 1 launch: one wave per column range)
  const int nacc = side == 0 ? left_tr16(nb) * nb : right_mc16(nb) * nb;
  return (size_t)wm * nacc * 4 * 64 * sizeof(double);
}

hipError_t pm_launch_16(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  const int RP = 16 * L.nb;
  if (!a.hpack || !a.hscale) return hipErrorInvalidValue;
  const bool bf = L.dtype == NNCP_BF16;
  PackArgs pa{a.krp.f[0], a.I1, a.I1pad, a.R, a.col0, RP, a.hpack, a.hscale};
  const int wm = a.wm;
  const bool fast = pm16_fast(L.side, a.IL, a.I1, L.nb);
  const bool mt = L.mper > 1;
  // variant = j1*100000 + bf16*10000 + side*1000 + nb*100 + mt*10 + fast
  const int variant =
      (L.j1 ? 100000 : 0) + (bf ? 10000 : 0) + L.side * 1000 + L.nb * 100 + (mt ? 10 : 0) + (fast ? 1 : 0);
  const void* k = kernel16(L.dtype, L.side, L.nb, L.j1, fast, mt, false);
  if (!k || (wm != 1 && wm != 4) || (L.j1 && wm != 4)) return hipErrorInvalidValue;
  size_t lds = L.lds_bytes;
  if (pm_16_reduce_lds(L.side, L.nb, wm) > lds) lds = pm_16_reduce_lds(L.side, L.nb, wm);
  if (lds > kPmMaxLds) return hipErrorInvalidValue;
  if (sk.rec) {
    KOp op{};
    op.kind = K_PACK16;
    op.variant = bf ? 1 : 0;
    op.gx = (unsigned)RP;
    op.gy = 1;
    op.u.pk = pa;
    hipError_t e = sink_record(sk, op);
    if (e != hipSuccess) return e;
    KOp pm{};
    pm.kind = K_PM_16;
    pm.variant = variant;
    pm.gx = (unsigned)L.mgroups;
    pm.gy = (unsigned)L.nsplit;
    pm.lds = (unsigned)lds;
    pm.u.pm = a;
    if (a.sctab) {
      e = pm_scale_table_record(L, a, sk);
      if (e != hipSuccess) return e;
    }
    return sink_record(sk, pm);
  }
  if (a.sctab) {
    hipError_t e = pm_scale_table_launch(L, a, sk.st);
    if (e != hipSuccess) return e;
  }
  {
    void* pargs[] = {(void*)&pa};
    hipError_t e = hipLaunchKernel(bf ? pm16_pack_kernel<NNCP_BF16>(false) : pm16_pack_kernel<NNCP_F16>(false),
                                   dim3(RP), dim3(256), pargs, 0, sk.st);
    if (e != hipSuccess) return e;
  }
  allow_big_lds(k);
  void* args[] = {(void*)&a};
  return hipLaunchKernel(k, dim3(L.mgroups, L.nsplit), dim3(NT), args, lds, sk.st);
}

const void* pm16_batch_kernel(int variant) {
  const int j1 = variant >= 100000 ? 1 : 0;
  const int dtype = ((variant / 10000) % 10) ? NNCP_BF16 : NNCP_F16;
  const int side = (variant / 1000) % 10, nb = (variant / 100) % 10;
  const void* k = kernel16(dtype, side, nb, j1, variant % 10, (variant / 10) % 10, true);
  if (k) allow_big_lds(k);
  return k;
}

const void* pm16_pack_batch_kernel(int variant) {
  return variant ? pm16_pack_kernel<NNCP_BF16>(true) : pm16_pack_kernel<NNCP_F16>(true);
}

}  // namespace nncpk
