// Batched 2D passes: the pipeline of Table 1 (steps 2-6) for many
// independent instances per launch, with 7-smooth padded lengths.
//
//   splat     one thread per source over the packed Y of all instances; the
//             instance is found by binary search in the source offsets.  The
//             sum of squared multiplicities that the validity threshold needs
//             is accumulated from the atomic's old value: adding a source to a
//             node holding m sources raises sum m^2 by 2m + 1.
//   finalize  Theta, S_max per instance.
//   row_r2c   rows of the count image -> half spectrum (packed complex
//             transform of length M_x/2 and the usual split of even/odd parts).
//   col_fused along y: forward transform of n_y nonzero rows, product with
//             the kernel spectra f, u_x, u_y (Table 1 step 4; eqs. SxSyconv),
//             inverse transform, rows y < n_y kept.
//   row_c2r   half spectrum -> real rows, fused with S = -tau log phi and the
//             gradient ratios (Sec. 2.3, Sec. 5), validity as in the single path.
#include <math.h>

#include "dt_batch.hpp"
#include "epilogue.hpp"

namespace dt {

__device__ __forceinline__ int batch_find(const int64_t* __restrict__ koff, int n, int64_t k) {
  int lo = 0, hi = n;   // koff[lo] <= k < koff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (koff[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int ceil_log2_count(int64_t K) {
  int e = 0;
  while (((int64_t)1 << e) < K) ++e;
  return e;
}

// ---------------------------------------------------------------------------
// Splat and validity scalars
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_batch_splat(const float* __restrict__ Y, int64_t K_total, BatchArgs a,
                                                     T* __restrict__ img) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int inst = -1;
  double inc = 0.0;
  if (k < K_total) {
    inst = batch_find(a.koff, a.n_inst, k);
    const BatchInst& I = a.inst[inst];
    const double y0 = (double)Y[2 * k], y1 = (double)Y[2 * k + 1];
    bool ok = isfinite(y0) && isfinite(y1);
    if (!ok) {
      atomicOr(a.err, kErrNonFinite);
    } else {
      const double q0 = floor((y0 - I.ox) / I.hx);
      const double q1 = floor((y1 - I.oy) / I.hy);
      ok = q0 >= 0.0 && q0 < (double)I.nx && q1 >= 0.0 && q1 < (double)I.ny;
      if (!ok) {
        atomicOr(a.err, kErrRange);
      } else {
        const int64_t Ki = a.koff[inst + 1] - a.koff[inst];
        const int eg = ceil_log2_count(Ki);
        const T cval = (T)ldexp(1.0, -eg);
        const int64_t lin = I.img_off + (int64_t)q0 + (int64_t)I.nx * (int64_t)q1;
        const T old = atomicAdd(&img[lin], cval);
        inc = 2.0 * ldexp((double)old, eg) + 1.0;
      }
    }
  }
  // one atomic per wave when the whole wave belongs to one instance
  const int first = __shfl(inst, 0);
  if (__all(inst == first) && first >= 0) {
    double s = inc;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(&a.scal[4 * first + 3], s);
  } else if (inst >= 0 && inc != 0.0) {
    atomicAdd(&a.scal[4 * inst + 3], inc);
  }
}

__global__ void __launch_bounds__(256) k_batch_finalize(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_inst) return;
  const double gl2 = sqrt(a.scal[4 * i + 3]);
  double theta = INFINITY, smax = INFINITY;   // no sources: S = +inf, zero gradient
  if (gl2 > 0.0) {
    theta = a.inst[i].theta_coef * gl2;
    smax = -a.inst[i].tau * log(theta);
  }
  a.scal[4 * i + 0] = theta;
  a.scal[4 * i + 1] = smax;
  a.scal[4 * i + 2] = gl2;
}

template <typename T> void launch_batch_splat(const float* Y, int64_t K_total, const BatchArgs& a, T* img,
                                              hipStream_t st) {
  if (K_total > 0) {
    const int64_t blocks = (K_total + 255) / 256;
    hipLaunchKernelGGL(k_batch_splat<T>, dim3((unsigned)blocks), dim3(256), 0, st, Y, K_total, a, img);
  }
}
void launch_batch_finalize(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_finalize, dim3((a.n_inst + 255) / 256), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// Row pass: count image rows -> half spectrum
// ---------------------------------------------------------------------------
template <typename T, int ECAP>
__global__ void __launch_bounds__(512) k_batch_row_r2c(BatchArgs a) {
  using V = Cx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const BatchBlock bb = a.blocks[blockIdx.x];
  const BatchInst* I = a.inst + bb.inst;
  const int N = I->sx, L = bb.count, LP = N + 1, nx = I->nx, pitch = I->pitch;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const T* img = (const T*)a.in + I->img_off + (int64_t)bb.first * nx;
  const V* twg = (const V*)a.tw + I->twx_off;
  V* tw = lds + L * LP;      // exp(-2 pi i m / M_x), m < M_x, staged for every stage
  for (int t = tid; t < 2 * N; t += nthr) tw[t] = twg[t];
  const FastDiv fN((uint32_t)N, I->m_sx), fH((uint32_t)(N + 1), I->m_sx1);
  for (int t = tid; t < L * N; t += nthr) {
    const int l = (int)fN.div((uint32_t)t), m = t - l * N;
    const T* src = img + (int64_t)l * nx;
    const T x0 = 2 * m < nx ? src[2 * m] : T(0);
    const T x1 = 2 * m + 1 < nx ? src[2 * m + 1] : T(0);
    lds[l * LP + m] = mk<V>(x0, x1);
  }
  __syncthreads();
  const MixedPlan& px = I->px;   // read per stage from the descriptor (no private copy)
  mixed_fft<T, 1, ECAP, false>(lds, N, FastDiv((uint32_t)L, (uint32_t)bb.magic), 1, LP, px, tw, 2, tid, nthr);
  V* out = (V*)a.out + I->spec_off + (int64_t)bb.first * pitch;
  const int H = N + 1;
  for (int t = tid; t < L * H; t += nthr) {
    const int l = (int)fH.div((uint32_t)t), k = t - l * H;
    const V zk = lds[l * LP + (k == N ? 0 : k)];
    const V zc = cconj(lds[l * LP + (k == 0 ? 0 : N - k)]);
    const V ev = cscale(cadd(zk, zc), T(0.5));
    const V od = cscale(mul_mi(csub(zk, zc)), T(0.5));
    out[(int64_t)l * pitch + k] = cadd(ev, cmul(tw[k], od));
  }
}

// ---------------------------------------------------------------------------
// Column pass along y: forward, kernel products, inverse, first n_y rows
// ---------------------------------------------------------------------------
template <typename T, int ECAP>
__global__ void __launch_bounds__(ECAP == 8 ? 1024 : 512) k_batch_col_fused(BatchArgs a) {
  using V = Cx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const BatchBlock bb = a.blocks[blockIdx.x];
  const BatchInst* I = a.inst + bb.inst;
  const int N = I->My, L = bb.count, ny = I->ny, pitch = I->pitch;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int NL = N * L;
  const FastDiv fL((uint32_t)L, (uint32_t)bb.magic);
  // two LDS buffers: the forward spectrum (kept) and the inverse work column
  V* spec = lds;
  V* work = lds + NL;
  V* twl = lds + 2 * NL;     // the instance's twiddles exp(-2 pi i m / M_y), read by every stage
  const V* in = (const V*)a.in + I->spec_off + bb.first;
  for (int t = tid; t < NL; t += nthr) {
    const int i = (int)fL.div((uint32_t)t), l = t - i * L;
    spec[t] = i < ny ? in[(int64_t)i * pitch + l] : mk<V>(T(0), T(0));
  }
  const V* twg = (const V*)a.tw + I->twy_off;
  for (int t = tid; t < N; t += nthr) twl[t] = twg[t];
  __syncthreads();
  const MixedPlan& py = I->py;
  const V* tw = twl;
  mixed_fft<T, 1, ECAP, true>(spec, N, fL, L, 1, py, tw, 1, tid, nthr);
  const T* tab = (const T*)a.tab + I->tab_off + bb.first;
  V* out = (V*)a.out + I->fused_off + bb.first;
  const int64_t ch_out = (int64_t)ny * pitch;
  for (int c = 0; c < a.C; ++c) {
    const T* tc = tab + c * I->tab_stride;
    const bool odd_y = c == 2;   // u_y is odd in y; u_x and u_y carry the factor -i
    for (int e = tid; e < NL; e += nthr) {
      const int i = (int)fL.div((uint32_t)e), l = e - i * L;
      const bool hi = 2 * i > N;
      T tv = tc[(int64_t)(hi ? N - i : i) * pitch + l];
      if (odd_y && hi) tv = -tv;
      const V z = cscale(spec[e], tv);
      work[e] = c == 0 ? z : mul_mi(z);
    }
    __syncthreads();
    mixed_fft<T, -1, ECAP, true>(work, N, fL, L, 1, py, tw, 1, tid, nthr);
    V* oc = out + c * ch_out;
    for (int t = tid; t < ny * L; t += nthr) {
      const int i = (int)fL.div((uint32_t)t), l = t - i * L;
      oc[(int64_t)i * pitch + l] = work[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Row pass: half spectrum -> real, fused with the epilogue
// ---------------------------------------------------------------------------
template <typename T, int ECAP>
__global__ void __launch_bounds__(512) k_batch_row_c2r_epi(BatchArgs a) {
  using V = Cx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const BatchBlock bb = a.blocks[blockIdx.x];
  const int ii = bb.inst;
  const BatchInst* I = a.inst + ii;
  const int N = I->sx, L = bb.count, C = a.C, LP = N + 1;
  const int nx = I->nx, ny = I->ny, pitch = I->pitch;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const V* in = (const V*)a.in + I->fused_off + (int64_t)bb.first * pitch;
  const V* twg = (const V*)a.tw + I->twx_off;
  V* tw = lds + L * C * LP;  // exp(-2 pi i m / M_x), m < M_x, staged for every stage
  for (int t = tid; t < 2 * N; t += nthr) tw[t] = twg[t];
  __syncthreads();
  const int64_t ch_in = (int64_t)ny * pitch;
  const FastDiv fN((uint32_t)N, I->m_sx), fC((uint32_t)C, C == kBatchChan ? fastdiv_magic(kBatchChan) : 0u),
      fX((uint32_t)nx, I->m_nx);
  for (int t = tid; t < L * C * N; t += nthr) {
    const int line = (int)fN.div((uint32_t)t), k = t - line * N;
    const int l = (int)fC.div((uint32_t)line), c = line - l * C;
    const V* src = in + c * ch_in + (int64_t)l * pitch;
    const V xk = src[k];
    const V xc = cconj(src[N - k]);
    const V ev = cadd(xk, xc);
    const V od = cmul(csub(xk, xc), cconj(tw[k]));
    lds[line * LP + k] = mk<V>(ev.x - od.y, ev.y + od.x);   // ev + i od
  }
  __syncthreads();
  const MixedPlan& px = I->pxi;   // read per stage from the descriptor (no private copy)
  mixed_fft<T, -1, ECAP, false>(lds, N, FastDiv((uint32_t)(L * C), (uint32_t)bb.magic), 1, LP, px, tw, 2, tid, nthr);
  const int64_t Ki = a.koff[ii + 1] - a.koff[ii];
  const int eg = ceil_log2_count(Ki);
  const T scale_phi = (T)ldexp(1.0, eg + I->e_f);
  const T su0 = (T)ldexp(1.0, I->e_u[0] - I->e_f);
  const T su1 = (T)ldexp(1.0, I->e_u[1] - I->e_f);
  const T theta = (T)a.scal[4 * ii + 0];
  const T smax = (T)a.scal[4 * ii + 1];
  const T tau = (T)I->tau;
  const T* ldr = reinterpret_cast<const T*>(lds);
  T* S = (T*)a.S;
  T* G = (T*)a.grad;
  const int64_t plane = (int64_t)nx * ny;
  for (int t = tid; t < L * nx; t += nthr) {
    const int l = (int)fX.div((uint32_t)t), x = t - l * nx;
    const int64_t node = (int64_t)(bb.first + l) * nx + x;
    const T cphi = ldr[(int64_t)(l * C) * 2 * LP + x];
    const T phi = cphi * scale_phi;
    const bool valid = phi >= theta;
    if (S) S[I->out_off + node] = valid ? -tau * epi_log(phi) : smax;
    if (G && C == kBatchChan) {
      const T inv = valid ? epi_rcp(cphi) : T(0);
      const T g0 = valid ? ldr[(int64_t)(l * C + 1) * 2 * LP + x] * inv * su0 : T(0);
      const T g1 = valid ? ldr[(int64_t)(l * C + 2) * 2 * LP + x] * inv * su1 : T(0);
      G[2 * I->out_off + node] = g0;
      G[2 * I->out_off + plane + node] = g1;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers: ECAP (elements per thread) picks the instantiation
// ---------------------------------------------------------------------------
#define DT_BATCH_DISPATCH(KER, T, a, n_blocks, nthr, ecap, lds, st)                                  \
  do {                                                                                                 \
    if ((n_blocks) <= 0) return true;                                                                  \
    if ((ecap) <= 8 && (nthr) <= 512)                                                                  \
      hipLaunchKernelGGL((KER<T, 8>), dim3(n_blocks), dim3(nthr), lds, st, a);                         \
    else if ((ecap) <= 16 && (nthr) <= 512)                                                            \
      hipLaunchKernelGGL((KER<T, 16>), dim3(n_blocks), dim3(nthr), lds, st, a);                        \
    else if ((ecap) <= 32 && (nthr) <= 512)                                                            \
      hipLaunchKernelGGL((KER<T, 32>), dim3(n_blocks), dim3(nthr), lds, st, a);                        \
    else                                                                                               \
      return false;                                                                                    \
    return true;                                                                                       \
  } while (0)

template <typename T> bool launch_batch_row_r2c(const BatchArgs& a, int n_blocks, int nthr, int ecap, size_t lds,
                                                hipStream_t st) {
  DT_BATCH_DISPATCH(k_batch_row_r2c, T, a, n_blocks, nthr, ecap, lds, st);
}
template <typename T> bool launch_batch_row_c2r_epi(const BatchArgs& a, int n_blocks, int nthr, int ecap,
                                                    size_t lds, hipStream_t st) {
  DT_BATCH_DISPATCH(k_batch_row_c2r_epi, T, a, n_blocks, nthr, ecap, lds, st);
}
template <typename T> bool launch_batch_col_fused(const BatchArgs& a, int n_blocks, int nthr, int ecap,
                                                  size_t lds, hipStream_t st) {
  if (n_blocks <= 0) return true;
  if (ecap <= 8 && nthr <= 1024)
    hipLaunchKernelGGL((k_batch_col_fused<T, 8>), dim3(n_blocks), dim3(nthr), lds, st, a);
  else if (ecap <= 16 && nthr <= 512)
    hipLaunchKernelGGL((k_batch_col_fused<T, 16>), dim3(n_blocks), dim3(nthr), lds, st, a);
  else if (ecap <= 32 && nthr <= 512)
    hipLaunchKernelGGL((k_batch_col_fused<T, 32>), dim3(n_blocks), dim3(nthr), lds, st, a);
  else
    return false;
  return true;
}

template <typename T> bool batch_set_lds_limit(int bytes) {
  const void* fns[] = {
      reinterpret_cast<const void*>(&k_batch_row_r2c<T, 8>),     reinterpret_cast<const void*>(&k_batch_row_r2c<T, 16>),
      reinterpret_cast<const void*>(&k_batch_row_r2c<T, 32>),    reinterpret_cast<const void*>(&k_batch_col_fused<T, 8>),
      reinterpret_cast<const void*>(&k_batch_col_fused<T, 16>),  reinterpret_cast<const void*>(&k_batch_col_fused<T, 32>),
      reinterpret_cast<const void*>(&k_batch_row_c2r_epi<T, 8>), reinterpret_cast<const void*>(&k_batch_row_c2r_epi<T, 16>),
      reinterpret_cast<const void*>(&k_batch_row_c2r_epi<T, 32>)};
  for (const void* f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return false;
  return true;
}

template void launch_batch_splat<float>(const float*, int64_t, const BatchArgs&, float*, hipStream_t);
template void launch_batch_splat<double>(const float*, int64_t, const BatchArgs&, double*, hipStream_t);
template bool launch_batch_row_r2c<float>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool launch_batch_row_r2c<double>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool launch_batch_col_fused<float>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool launch_batch_col_fused<double>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool launch_batch_row_c2r_epi<float>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool launch_batch_row_c2r_epi<double>(const BatchArgs&, int, int, int, size_t, hipStream_t);
template bool batch_set_lds_limit<float>(int);
template bool batch_set_lds_limit<double>(int);

}  // namespace dt
