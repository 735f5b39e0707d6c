// Population control of a system's walkers (comb; pair branching) and weighted statistics of
// the energy records (Sec. "Computational Details": comb population control, and pair branching
// for Theta <= 0.25; estimators are weight-averaged over walkers, Sec. "Finite-Temperature
// AFQMC in the Grand Canonical Ensemble").  Both methods copy whole walkers; which walkers and
// how often follows their published definitions:
//   comb: total weight T, one uniform u; teeth at (k + u) T / W, k < W; walker i takes the
//         teeth in [c_{i-1}, c_i) (c = running sums from walker 0), every copy weighs T / W;
//   pair branch: the p-th heaviest walker pairs with the p-th lightest while the heavy one
//         weighs more than 2 T/W or the light one less than T/(2W); with probability
//         w_l / (w_l + w_s) (uniform u_p) both slots become the heavy walker, else the light
//         one, each with weight (w_l + w_s) / 2.
// Slots: a walker that keeps a copy keeps its slot; further copies fill the slots of walkers
// that keep none, in ascending order, taken by the copies in tooth order; so every copy reads a
// slot that is not written.  Weights are w_i = exp(ln w_i - max ln w) over live walkers, 0 for
// killed or numeric ones; ties in the weight order go to the lower index.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int NT = 256;

FT_DEV double block_max_256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  const double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return t;
}

// One workgroup: parent[j] = walker copied into slot j, newlogw[j] its new ln w.
// Dynamic LDS: w [W] double, c [W] double, a [W] int, b [W] int.
__global__ __launch_bounds__(NT) void pop_select_kernel(const double* logw, const int* status, int W, int method,
                                                        const double* u, int* parent, double* newlogw) {
  extern __shared__ char dyn[];
  double* w = (double*)dyn;
  double* c = w + W;
  int* a = (int*)(c + W);
  int* b = a + W;
  __shared__ double red[4];
  __shared__ int any_live;
  double mx = -INFINITY;
  for (int i = threadIdx.x; i < W; i += NT)
    if (status[i] == 0 && isfinite(logw[i])) mx = fmax(mx, logw[i]);
  mx = block_max_256(mx, red);
  if (threadIdx.x == 0) any_live = mx > -INFINITY;
  for (int i = threadIdx.x; i < W; i += NT) {
    const bool live = status[i] == 0 && isfinite(logw[i]);
    w[i] = live ? exp(logw[i] - mx) : 0.0;
    parent[i] = i;
    newlogw[i] = logw[i];
  }
  __syncthreads();
  if (!any_live) return;
  if (threadIdx.x == 0) {                      // running sums, walker 0 upwards
    double acc = 0.0;
    for (int i = 0; i < W; ++i) { acc += w[i]; c[i] = acc; }
  }
  __syncthreads();
  const double total = c[W - 1];
  if (method == 0) {
    if (threadIdx.x != 0) return;
    const double step = total / W;
    int last = W - 1;
    while (last > 0 && !(w[last] > 0.0)) --last;
    for (int i = 0; i < W; ++i) a[i] = 0;     // copies per walker
    int i = 0;
    for (int k = 0; k < W; ++k) {             // b[k] = owner of tooth k
      const double t = ((double)k + u[0]) * step;
      while (i < W && !(c[i] > t)) ++i;
      const int owner = i < W ? i : last;
      a[owner] += 1;
      b[k] = owner;
      if (i > W - 1) i = W - 1;
    }
    int f = 0;                                // next free slot
    for (int k = 0; k < W; ++k) {
      const int owner = b[k];
      if (k > 0 && b[k - 1] == owner) {        // a further copy of the same walker (teeth are ordered)
        while (a[f] != 0) ++f;
        parent[f] = owner;
        ++f;
      }
    }
    const double lw = log(step) + mx;
    for (int j = 0; j < W; ++j) newlogw[j] = lw;
    return;
  }
  // pair branch: ranks in descending (a) and ascending (b) weight order, ties to the lower index
  for (int i = threadIdx.x; i < W; i += NT) {
    const double wi = w[i];
    int rd = 0, ra = 0;
    for (int j = 0; j < W; ++j) {
      const double wj = w[j];
      rd += (wj > wi || (wj == wi && j < i)) ? 1 : 0;
      ra += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
    }
    a[rd] = i;
    b[ra] = i;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double wbar = total / W;
  for (int p = 0; p < W / 2; ++p) {
    const int l = a[p], s = b[p];
    if (!(w[l] > 2.0 * wbar || w[s] < 0.5 * wbar)) break;
    const double tot = w[l] + w[s];
    if (u[p] * tot < w[l]) parent[s] = l;
    else parent[l] = s;
    const double lw = log(0.5 * tot) + mx;
    newlogw[l] = lw;
    newlogw[s] = lw;
  }
}

// Copy the walker state of parent[j] into slot j (j != parent[j]) and set every ln w:
// Y, T^{-1}, G ([ld][ld] each; and the constraint's G when it is a separate buffer), D [ld],
// r [NQ] (and the force bias's r when separate); ln det(I + A), ln det T, status.
constexpr int POP_CHUNK = 8192;
__global__ __launch_bounds__(NT) void pop_copy_kernel(SysDev s, const int* parent, const double* newlogw, int chunks,
                                                      int nmat) {
  const int j = blockIdx.x / chunks, ch = blockIdx.x - j * chunks;
  if (j >= s.W) return;
  const int src = parent[j];
  if (ch == 0 && threadIdx.x == 0) s.logw[j] = newlogw[j];
  if (src == j) return;
  const long long mat = s.mat_stride;
  const long long e0 = (long long)ch * POP_CHUNK, e1 = min(e0 + POP_CHUNK, nmat * mat);
  for (long long e = e0 + threadIdx.x; e < e1; e += NT) {
    const int m = (int)(e / mat);
    const long long o = e - m * mat;
    double2* base = m == 0 ? s.Y : (m == 1 ? s.Ti : (m == 2 ? s.G : s.Gt));
    base[(long long)j * mat + o] = base[(long long)src * mat + o];
  }
  if (ch == chunks - 1) {
    for (int i = threadIdx.x; i < s.ld; i += NT) s.D[(long long)j * s.ld + i] = s.D[(long long)src * s.ld + i];
    for (int q = threadIdx.x; q < s.NQ; q += NT) s.r[(long long)j * s.NQ + q] = s.r[(long long)src * s.NQ + q];
    if (s.rb != s.r)
      for (int q = threadIdx.x; q < s.NQ; q += NT) s.rb[(long long)j * s.NQ + q] = s.rb[(long long)src * s.NQ + q];
    if (threadIdx.x == 0) {
      s.ell[j] = s.ell[src];
      s.lndetT[j] = s.lndetT[src];
      s.status[j] = s.status[src];
    }
  }
}

// Weighted statistics of every energy record (one workgroup per record): Re<E>, its standard
// error sqrt(sum w^2 (Re E - Re<E>)^2) / sum w (delta method for the ratio estimator), Re<N>
// and its standard error, sum w / max w, ln max w, the effective walker count
// (sum w)^2 / sum w^2 and the number of live walkers.  Then, in avg, the averages over the
// records that have live walkers of Re<E> and Re<N> (the time-slice average of the global
// estimate) and the number of such records.
constexpr int NSTAT = 8;
__global__ __launch_bounds__(NT) void record_stats_kernel(const double2* rec_E, const double* rec_logw,
                                                          const int* rec_status, int W, int nrec, double* stats) {
  __shared__ double red[8];
  const int r = blockIdx.x;
  if (r >= nrec) return;
  const double2* E = rec_E + (long long)r * W * 4;
  const double* lw = rec_logw + (long long)r * W;
  const int* st = rec_status + (long long)r * W;
  double mx = -INFINITY;
  for (int i = threadIdx.x; i < W; i += NT)
    if (st[i] == 0 && isfinite(lw[i])) mx = fmax(mx, lw[i]);
  mx = block_max_256(mx, red);
  double sw = 0.0, sw2 = 0.0, se = 0.0, sn = 0.0, nl = 0.0;
  for (int i = threadIdx.x; i < W; i += NT)
    if (st[i] == 0 && isfinite(lw[i])) {
      const double wi = exp(lw[i] - mx);
      sw += wi; sw2 += wi * wi; se += wi * E[(long long)i * 4 + 2].x; sn += wi * E[(long long)i * 4 + 3].x; nl += 1.0;
    }
  sw = block_sum_256(sw, red); sw2 = block_sum_256(sw2, red);
  se = block_sum_256(se, red); sn = block_sum_256(sn, red); nl = block_sum_256(nl, red);
  const double me = sw > 0.0 ? se / sw : NAN, mn = sw > 0.0 ? sn / sw : NAN;
  double ve = 0.0, vn = 0.0;
  for (int i = threadIdx.x; i < W; i += NT)
    if (st[i] == 0 && isfinite(lw[i])) {
      const double wi = exp(lw[i] - mx);
      const double de = E[(long long)i * 4 + 2].x - me, dn = E[(long long)i * 4 + 3].x - mn;
      ve += wi * wi * de * de; vn += wi * wi * dn * dn;
    }
  ve = block_sum_256(ve, red); vn = block_sum_256(vn, red);
  if (threadIdx.x == 0) {
    double* o = stats + (long long)r * NSTAT;
    o[0] = me; o[1] = sw > 0.0 ? sqrt(ve) / sw : NAN; o[2] = mn; o[3] = sw > 0.0 ? sqrt(vn) / sw : NAN;
    o[4] = sw; o[5] = mx; o[6] = sw > 0.0 ? sw * sw / sw2 : 0.0; o[7] = nl;
  }
}

__global__ void record_average_kernel(const double* stats, int nrec, double* avg) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double e = 0.0, n = 0.0, cnt = 0.0;
  for (int r = 0; r < nrec; ++r)
    if (stats[(long long)r * NSTAT + 7] > 0.0) { e += stats[(long long)r * NSTAT]; n += stats[(long long)r * NSTAT + 2]; cnt += 1.0; }
  avg[0] = cnt > 0.0 ? e / cnt : NAN;
  avg[1] = cnt > 0.0 ? n / cnt : NAN;
  avg[2] = cnt;
}

}  // namespace

size_t pop_select_lds(int W) { return (size_t)W * (2 * sizeof(double) + 2 * sizeof(int)); }

hipError_t launch_population_control(const SysDev& s, int method, const double* u, int* parent, double* newlogw,
                                     hipStream_t st) {
  const size_t lds = pop_select_lds(s.W);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  pop_select_kernel<<<1, NT, lds, st>>>(s.logw, s.status, s.W, method, u, parent, newlogw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nmat = s.Gt != s.G ? 4 : 3;
  const int chunks = (int)((nmat * s.mat_stride + POP_CHUNK - 1) / POP_CHUNK);
  pop_copy_kernel<<<s.W * chunks, NT, 0, st>>>(s, parent, newlogw, chunks, nmat);
  return hipGetLastError();
}

hipError_t launch_record_stats(const SysDev& s, int nrec, double* stats, double* avg, hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  record_stats_kernel<<<nrec, NT, 0, st>>>(s.rec_E, s.rec_logw, s.rec_status, s.rec_W, nrec, stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !avg) return e;
  record_average_kernel<<<1, 64, 0, st>>>(stats, nrec, avg);
  return hipGetLastError();
}
