// Direct volume rendering of one block's INR by sample streaming (gfx950).
//
// Ray marching is split into separate launches per round, so that the INR
// inference between them runs on large, dense batches of samples (the
// sample-streaming organisation of Sec. IV):
//   k_ray_init : pinhole ray through each pixel center, intersection with the
//                block's unit cube, accumulators cleared, hit rays listed;
//   k_ray_gen  : samples k_base .. k_base + S - 1 of every active ray ->
//                coordinates for the inference kernels;
//   (encode + MLP inference over the batch, as dvnr_sample)
//   k_ray_shade: transfer function, opacity correction and front-to-back
//                compositing of each ray's S samples in order; rays that
//                neither left the cube nor reached the opacity limit are
//                appended to the next round's list.
// Ray setup and sample positions use round-to-nearest intrinsics in a fixed
// operation order (no contraction into FMA): the number of samples of a ray
// is an integer decided by these values.
#include "dvnr_device.h"

namespace dvnrk {

__device__ __forceinline__ float dot3_rn(float ax, float ay, float az, float bx, float by, float bz) {
  return fadd_nc(fadd_nc(fmul_nc(ax, bx), fmul_nc(ay, by)), fmul_nc(az, bz));
}

__device__ __forceinline__ void normalize_rn(float* v) {
  const float n = __fsqrt_rn(dot3_rn(v[0], v[1], v[2], v[0], v[1], v[2]));
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = __fdiv_rn(v[a], n);
}

__device__ __forceinline__ void cross_rn(const float* a, const float* b, float* c) {
  c[0] = fsub_nc(fmul_nc(a[1], b[2]), fmul_nc(a[2], b[1]));
  c[1] = fsub_nc(fmul_nc(a[2], b[0]), fmul_nc(a[0], b[2]));
  c[2] = fsub_nc(fmul_nc(a[0], b[1]), fmul_nc(a[1], b[0]));
}

__global__ __launch_bounds__(256) void k_ray_init(RayCamera cam, int width, int height, float* __restrict__ dirs,
                                                  float* __restrict__ t01, float* __restrict__ rgba,
                                                  int32_t* __restrict__ active, int32_t* __restrict__ counter) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= width * height) return;
  // camera frame: f = normalize(center - eye), r = normalize(f x up), u = r x f
  float fw[3], rt[3], uu[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) fw[a] = fsub_nc(cam.center[a], cam.eye[a]);
  normalize_rn(fw);
  cross_rn(fw, cam.up, rt);
  normalize_rn(rt);
  cross_rn(rt, fw, uu);
  const float aspect = __fdiv_rn((float)width, (float)height);
  const int i = p % width, j = p / width;
  const float px = fmul_nc(fmul_nc(fsub_nc(__fdiv_rn(fmul_nc(2.0f, fadd_nc((float)i, 0.5f)), (float)width),
                                                 1.0f),
                                       cam.tan_h),
                             aspect);
  const float py =
      fmul_nc(fsub_nc(1.0f, __fdiv_rn(fmul_nc(2.0f, fadd_nc((float)j, 0.5f)), (float)height)), cam.tan_h);
  float d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = fadd_nc(fadd_nc(fw[a], fmul_nc(px, rt[a])), fmul_nc(py, uu[a]));
  const float n = __fsqrt_rn(dot3_rn(d[0], d[1], d[2], d[0], d[1], d[2]));
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = __fdiv_rn(d[a], n);
  // slab intersection with [0,1]^3
  float t0 = 0.0f, t1 = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float inv = __fdiv_rn(1.0f, d[a]);
    const float ta = fmul_nc(fsub_nc(0.0f, cam.eye[a]), inv);
    const float tb = fmul_nc(fsub_nc(1.0f, cam.eye[a]), inv);
    t0 = fmaxf(t0, fminf(ta, tb));
    t1 = fminf(t1, fmaxf(ta, tb));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) dirs[3 * p + a] = d[a];
  t01[2 * p] = t0;
  t01[2 * p + 1] = t1;
#pragma unroll
  for (int c = 0; c < 4; ++c) rgba[4 * p + c] = 0.0f;
  if (t1 > t0) active[atomicAdd(counter, 1)] = p;
}

// Sample position t_k = t0 + (k + 1/2) dt; the sample exists iff t_k < t1.
__device__ __forceinline__ float sample_t(float t0, int k, float dt) {
  return fadd_nc(t0, fmul_nc(fadd_nc((float)k, 0.5f), dt));
}

__global__ __launch_bounds__(256) void k_ray_gen(RayCamera cam, const int32_t* __restrict__ active, int n_rays,
                                                 int k_base, int S, float dt, const float* __restrict__ dirs,
                                                 const float* __restrict__ t01, float* __restrict__ coords) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n_rays * S) return;
  const int jj = (int)(q / n_rays), r = (int)(q % n_rays);  // sample-major: shading reads coalesced
  const int p = active[r];
  const float tk = sample_t(t01[2 * p], k_base + jj, dt);
  const bool ok = tk < t01[2 * p + 1];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    coords[3 * q + a] = ok ? fadd_nc(cam.eye[a], fmul_nc(tk, dirs[3 * p + a])) : 0.5f;
}

// One lane per ray; values[jj * n_rays + r] is the de-normalized INR output of
// sample k_base + jj of active ray r (sample-major, so a wave's reads of one
// sample index are contiguous).
__global__ __launch_bounds__(256) void k_ray_shade(const int32_t* __restrict__ active, int n_rays, int k_base, int S,
                                                   float dt, float opacity_exp, float alpha_stop,
                                                   const float* __restrict__ t01, const float* __restrict__ values,
                                                   const float* __restrict__ tf, int n_tf, float tf_lo,
                                                   float tf_inv_range, float* __restrict__ rgba,
                                                   int32_t* __restrict__ next, int32_t* __restrict__ next_count) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  const int p = active[r];
  const float t0 = t01[2 * p], t1 = t01[2 * p + 1];
  float C0 = rgba[4 * p], C1 = rgba[4 * p + 1], C2 = rgba[4 * p + 2], A = rgba[4 * p + 3];
  bool done = false;
  for (int jj = 0; jj < S && !done; ++jj) {
    if (!(sample_t(t0, k_base + jj, dt) < t1)) {
      done = true;
      break;
    }
    const float v = values[(int64_t)jj * n_rays + r];
    const float s = fminf(fmaxf((v - tf_lo) * tf_inv_range, 0.0f), 1.0f) * (float)(n_tf - 1);
    const int i = min((int)floorf(s), n_tf - 2);
    const float w = s - (float)i;
    const float4 a = reinterpret_cast<const float4*>(tf)[i];
    const float4 b = reinterpret_cast<const float4*>(tf)[i + 1];
    const float op = fminf(fmaxf(a.w + w * (b.w - a.w), 0.0f), 1.0f);
    const float alpha = 1.0f - powf(1.0f - op, opacity_exp);
    const float wgt = (1.0f - A) * alpha;
    C0 += wgt * (a.x + w * (b.x - a.x));
    C1 += wgt * (a.y + w * (b.y - a.y));
    C2 += wgt * (a.z + w * (b.z - a.z));
    A += wgt;
    if (A >= alpha_stop) done = true;
  }
  rgba[4 * p] = C0;
  rgba[4 * p + 1] = C1;
  rgba[4 * p + 2] = C2;
  rgba[4 * p + 3] = A;
  if (!done) next[atomicAdd(next_count, 1)] = p;
}

hipError_t launch_ray_init(const RayCamera& cam, int width, int height, float* dirs, float* t01, float* rgba,
                           int32_t* active, int32_t* counter, hipStream_t s) {
  const int n = width * height;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ray_init, dim3((n + 255) / 256), dim3(256), 0, s, cam, width, height, dirs, t01, rgba, active,
                     counter);
  return hipGetLastError();
}

hipError_t launch_ray_gen(const RayCamera& cam, const int32_t* active, int n_rays, int k_base, int S, float dt,
                          const float* dirs, const float* t01, float* coords, hipStream_t s) {
  const int64_t n = (int64_t)n_rays * S;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ray_gen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cam, active, n_rays, k_base, S,
                     dt, dirs, t01, coords);
  return hipGetLastError();
}

hipError_t launch_ray_shade(const int32_t* active, int n_rays, int k_base, int S, float dt, float opacity_exp,
                            float alpha_stop, const float* t01, const float* values, const float* tf, int n_tf,
                            float tf_lo, float tf_inv_range, float* rgba, int32_t* next, int32_t* next_count,
                            hipStream_t s) {
  if (n_rays <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ray_shade, dim3((n_rays + 255) / 256), dim3(256), 0, s, active, n_rays, k_base, S, dt,
                     opacity_exp, alpha_stop, t01, values, tf, n_tf, tf_lo, tf_inv_range, rgba, next, next_count);
  return hipGetLastError();
}

}  // namespace dvnrk
