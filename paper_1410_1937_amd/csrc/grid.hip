// libnfa: stretched grid metrics and immersed-body geometry.
//
// Gridding section: a tensor-product grid given by its face coordinates.
// Enforcement of Body Boundary Conditions: fractional face areas and cell
// fractions of the fluid region psi > 0, active set, and merging of small
// cut cells with the neighbour along the steepest gradient of psi.
//
// The sampling kernels evaluate the bilinear / trilinear interpolants in a
// fixed operation order with FP contraction disabled (this file is built
// with -ffp-contract=off), so fractions are exactly reproducible.
#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "device_util.h"
#include "nfa_internal.h"

namespace nfa {
namespace {

// Share of S*S midpoint samples where the bilinear interpolant is > 0;
// (s along the first local axis, t along the second).  If every corner is
// > 0 (<= 0) every sample is, since all weights are strictly positive.
__device__ double bilinear_fraction(double c00, double c10, double c01, double c11, int S) {
  if (c00 > 0 && c10 > 0 && c01 > 0 && c11 > 0) return 1.0;
  if (c00 <= 0 && c10 <= 0 && c01 <= 0 && c11 <= 0) return 0.0;
  int cnt = 0;
  for (int tt = 0; tt < S; ++tt) {
    const double t = (tt + 0.5) / S;
    for (int ss = 0; ss < S; ++ss) {
      const double s = (ss + 0.5) / S;
      const double w00 = (1.0 - s) * (1.0 - t);
      const double w10 = s * (1.0 - t);
      const double w01 = (1.0 - s) * t;
      const double w11 = s * t;
      const double v = ((w00 * c00 + w10 * c10) + w01 * c01) + w11 * c11;
      cnt += v > 0;
    }
  }
  return (double)cnt / (double)(S * S);
}

__device__ __forceinline__ double node(const double* psi, int nx, int ny, int k, int j, int i) {
  return psi[((long long)k * (ny + 1) + j) * (nx + 1) + i];
}

__global__ void k_face_frac_x(int nx, int ny, int nz, const double* psi, int S, double* out) {
  const long long n = (long long)nz * ny * (nx + 1);
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    if (!psi) { out[f] = 1.0; continue; }
    const int i = (int)(f % (nx + 1));
    const long long r = f / (nx + 1);
    const int j = (int)(r % ny), k = (int)(r / ny);
    out[f] = bilinear_fraction(node(psi, nx, ny, k, j, i), node(psi, nx, ny, k, j + 1, i),
                               node(psi, nx, ny, k + 1, j, i), node(psi, nx, ny, k + 1, j + 1, i), S);
  }
}

__global__ void k_face_frac_y(int nx, int ny, int nz, const double* psi, int S, double* out) {
  const long long n = (long long)nz * (ny + 1) * nx;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    if (!psi) { out[f] = 1.0; continue; }
    const int i = (int)(f % nx);
    const long long r = f / nx;
    const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
    out[f] = bilinear_fraction(node(psi, nx, ny, k, j, i), node(psi, nx, ny, k, j, i + 1),
                               node(psi, nx, ny, k + 1, j, i), node(psi, nx, ny, k + 1, j, i + 1), S);
  }
}

__global__ void k_face_frac_z(int nx, int ny, int nz, const double* psi, int S, double* out) {
  const long long n = (long long)(nz + 1) * ny * nx;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    if (!psi) { out[f] = 1.0; continue; }
    const int i = (int)(f % nx);
    const long long r = f / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    out[f] = bilinear_fraction(node(psi, nx, ny, k, j, i), node(psi, nx, ny, k, j, i + 1),
                               node(psi, nx, ny, k, j + 1, i), node(psi, nx, ny, k, j + 1, i + 1), S);
  }
}

// Share of S^3 samples where the trilinear interpolant is > 0.  Corner order
// (a,b,c) with a (x) fastest; weight (wx_a * wy_b) * wz_c; summed in order.
__global__ void k_cell_frac(int nx, int ny, int nz, const double* psi, int S, double* out) {
  const long long n = (long long)nz * ny * nx;
  for (long long cidx = blockIdx.x * (long long)blockDim.x + threadIdx.x; cidx < n;
       cidx += (long long)gridDim.x * blockDim.x) {
    if (!psi) { out[cidx] = 1.0; continue; }
    const int i = (int)(cidx % nx);
    const long long r = cidx / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    double cm[8];
    bool allpos = true, allneg = true;
    int idx = 0;
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const double v = node(psi, nx, ny, k + c, j + b, i + a);
          cm[idx++] = v;
          allpos = allpos && (v > 0);
          allneg = allneg && (v <= 0);
        }
    if (allpos) { out[cidx] = 1.0; continue; }
    if (allneg) { out[cidx] = 0.0; continue; }
    int cnt = 0;
    for (int uu = 0; uu < S; ++uu) {
      const double u = (uu + 0.5) / S;
      const double wz[2] = {1.0 - u, u};
      for (int tt = 0; tt < S; ++tt) {
        const double t = (tt + 0.5) / S;
        const double wy[2] = {1.0 - t, t};
        for (int ss = 0; ss < S; ++ss) {
          const double s = (ss + 0.5) / S;
          const double wx[2] = {1.0 - s, s};
          double val = 0.0;
          int q = 0;
          for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
              for (int a = 0; a < 2; ++a) {
                const double term = ((wx[a] * wy[b]) * wz[c]) * cm[q];
                val = (q == 0) ? term : val + term;
                ++q;
              }
          cnt += val > 0;
        }
      }
    }
    out[cidx] = (double)cnt / (double)(S * S * S);
  }
}

// Active iff wet (fraction > 0) and some open coupling exists.
__global__ void k_active(int nx, int ny, int nz, const double* fx, const double* fy,
                         const double* fz, const double* vf, int b0, int b1, int b2, int b3, int b4,
                         int b5, unsigned char* act) {
  const long long n = (long long)nz * ny * nx;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const long long plane = (long long)nx * ny;
    bool wet = vf[c] > 0;
    bool cp = false;
    const long long xf = ((long long)k * ny + j) * (nx + 1) + i;
    const long long yf = ((long long)k * (ny + 1) + j) * nx + i;
    const long long zf = c;
    if (i > 0) cp |= fx[xf] > 0 && vf[c - 1] > 0; else cp |= b0 && fx[xf] > 0;
    if (i < nx - 1) cp |= fx[xf + 1] > 0 && vf[c + 1] > 0; else cp |= b1 && fx[xf + 1] > 0;
    if (j > 0) cp |= fy[yf] > 0 && vf[c - nx] > 0; else cp |= b2 && fy[yf] > 0;
    if (j < ny - 1) cp |= fy[yf + nx] > 0 && vf[c + nx] > 0; else cp |= b3 && fy[yf + nx] > 0;
    if (k > 0) cp |= fz[zf] > 0 && vf[c - plane] > 0; else cp |= b4 && fz[zf] > 0;
    if (k < nz - 1) cp |= fz[zf + plane] > 0 && vf[c + plane] > 0; else cp |= b5 && fz[zf + plane] > 0;
    act[c] = (wet && cp) ? 1 : 0;
  }
}

// open area = fraction * (touching cells active) * full face area
__global__ void k_open_x(int nx, int ny, int nz, const double* frac, const unsigned char* act,
                         const double* dy, const double* dz, double* out) {
  const long long n = (long long)nz * ny * (nx + 1);
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(f % (nx + 1));
    const long long r = f / (nx + 1);
    const int j = (int)(r % ny), k = (int)(r / ny);
    const long long c = ((long long)k * ny + j) * nx + i;
    double o = frac[f];
    if (i < nx) o *= act[c] ? 1.0 : 0.0;
    if (i > 0) o *= act[c - 1] ? 1.0 : 0.0;
    out[f] = o * (dz[k] * dy[j]);
  }
}
__global__ void k_open_y(int nx, int ny, int nz, const double* frac, const unsigned char* act,
                         const double* dx, const double* dz, double* out) {
  const long long n = (long long)nz * (ny + 1) * nx;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(f % nx);
    const long long r = f / nx;
    const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
    const long long c = ((long long)k * ny + j) * nx + i;
    double o = frac[f];
    if (j < ny) o *= act[c] ? 1.0 : 0.0;
    if (j > 0) o *= act[c - nx] ? 1.0 : 0.0;
    out[f] = o * (dz[k] * dx[i]);
  }
}
__global__ void k_open_z(int nx, int ny, int nz, const double* frac, const unsigned char* act,
                         const double* dx, const double* dy, double* out) {
  const long long n = (long long)(nz + 1) * ny * nx;
  const long long plane = (long long)nx * ny;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(f % nx);
    const long long r = f / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    double o = frac[f];
    if (k < nz) o *= act[f] ? 1.0 : 0.0;
    if (k > 0) o *= act[f - plane] ? 1.0 : 0.0;
    out[f] = o * (dy[j] * dx[i]);
  }
}

// Merge target of a small active cell: steepest |grad psi| axis (ties to the
// lower axis), toward larger psi, through an open interior face; -1 if none.
__global__ void k_merge_target(int nx, int ny, int nz, const double* psi, const double* vf,
                               const unsigned char* act, const double* ox, const double* oy,
                               const double* oz, const double* dx, const double* dy,
                               const double* dz, double theta, int* target) {
  const long long n = (long long)nz * ny * nx;
  const long long plane = (long long)nx * ny;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    target[c] = -1;
    if (!act[c] || !(vf[c] < theta)) continue;
    const int i = (int)(c % nx);
    const long long r = c / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    double P[2][2][2];
    for (int cc = 0; cc < 2; ++cc)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) P[cc][b][a] = node(psi, nx, ny, k + cc, j + b, i + a);
    double g[3];
    g[0] = ((((P[0][0][1] - P[0][0][0]) + (P[0][1][1] - P[0][1][0])) + (P[1][0][1] - P[1][0][0])) +
            (P[1][1][1] - P[1][1][0])) * 0.25 / dx[i];
    g[1] = ((((P[0][1][0] - P[0][0][0]) + (P[0][1][1] - P[0][0][1])) + (P[1][1][0] - P[1][0][0])) +
            (P[1][1][1] - P[1][0][1])) * 0.25 / dy[j];
    g[2] = ((((P[1][0][0] - P[0][0][0]) + (P[1][0][1] - P[0][0][1])) + (P[1][1][0] - P[0][1][0])) +
            (P[1][1][1] - P[0][1][1])) * 0.25 / dz[k];
    int order[3] = {0, 1, 2};
    // stable sort by descending |g|
    for (int a = 1; a < 3; ++a) {
      int v = order[a], b = a - 1;
      while (b >= 0 && fabs(g[order[b]]) < fabs(g[v])) { order[b + 1] = order[b]; --b; }
      order[b + 1] = v;
    }
    for (int q = 0; q < 3; ++q) {
      const int d = order[q];
      if (g[d] == 0.0) continue;
      const int s = g[d] > 0 ? 1 : -1;
      long long t;
      if (d == 0) {
        const int fi = i + (s > 0 ? 1 : 0);
        if (fi == 0 || fi == nx || !(ox[((long long)k * ny + j) * (nx + 1) + fi] > 0)) continue;
        t = c + s;
      } else if (d == 1) {
        const int fj = j + (s > 0 ? 1 : 0);
        if (fj == 0 || fj == ny || !(oy[((long long)k * (ny + 1) + fj) * nx + i] > 0)) continue;
        t = c + (long long)s * nx;
      } else {
        const int fk = k + (s > 0 ? 1 : 0);
        if (fk == 0 || fk == nz || !(oz[(long long)fk * plane + (long long)j * nx + i] > 0)) continue;
        t = c + (long long)s * plane;
      }
      target[c] = (int)t;
      break;
    }
  }
}

__global__ void k_reduced_init(long long n, const unsigned char* act, unsigned char* red, int* root) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    red[c] = act[c];
    root[c] = act[c] ? (int)c : -1;
  }
}

__global__ void k_reduced_slaves(int ns, const int* s_cell, const int* s_root, unsigned char* red,
                                 int* root) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += gridDim.x * blockDim.x) {
    red[s_cell[t]] = 0;
    root[s_cell[t]] = s_root[t];
  }
}

void axis_metrics(const double* f, int n, std::vector<double>& fv, std::vector<double>& d,
                  std::vector<double>& h) {
  fv.assign(f, f + n + 1);
  d.resize(n);
  for (int i = 0; i < n; ++i) d[i] = f[i + 1] - f[i];
  std::vector<double> c(n);
  for (int i = 0; i < n; ++i) c[i] = 0.5 * (f[i] + f[i + 1]);
  h.resize(n + 1);
  for (int i = 1; i < n; ++i) h[i] = c[i] - c[i - 1];
  h[0] = 0.5 * d[0];
  h[n] = 0.5 * d[n - 1];
}

// Denominators of the central differences of the interface normals: the
// distance between the centres either side of each cell, with a ghost centre
// mirrored across each boundary face.
std::vector<double> normal_den(const std::vector<double>& f) {
  const int n = (int)f.size() - 1;
  std::vector<double> cg(n + 2), den(n);
  for (int i = 0; i < n; ++i) cg[i + 1] = 0.5 * (f[i] + f[i + 1]);
  cg[0] = 2.0 * f[0] - cg[1];
  cg[n + 1] = 2.0 * f[n] - cg[n];
  for (int i = 0; i < n; ++i) den[i] = cg[i + 2] - cg[i];
  return den;
}

hipError_t upload(DevBuf& b, const std::vector<double>& v) {
  hipError_t e = b.alloc(v.size() * sizeof(double));
  if (e != hipSuccess) return e;
  return hipMemcpy(b.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
}

template <class T>
hipError_t upload_vec(DevBuf& b, const std::vector<T>& v) {
  hipError_t e = b.alloc(std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

nfa_status compute_body(Grid& g, const double* psi, double theta, int S, hipStream_t s) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long n = g.n;
  const int nb = blocks_for(std::max(std::max(g.nfx(), g.nfy()), g.nfz()));
  k_face_frac_x<<<nb, kBlock, 0, s>>>(nx, ny, nz, psi, S, g.frac_x.as<double>());
  k_face_frac_y<<<nb, kBlock, 0, s>>>(nx, ny, nz, psi, S, g.frac_y.as<double>());
  k_face_frac_z<<<nb, kBlock, 0, s>>>(nx, ny, nz, psi, S, g.frac_z.as<double>());
  k_cell_frac<<<nb, kBlock, 0, s>>>(nx, ny, nz, psi, S, g.vfrac.as<double>());
  k_active<<<nb, kBlock, 0, s>>>(nx, ny, nz, g.frac_x.as<double>(), g.frac_y.as<double>(),
                                 g.frac_z.as<double>(), g.vfrac.as<double>(), g.bc[0], g.bc[1],
                                 g.bc[2], g.bc[3], g.bc[4], g.bc[5], g.active.as<unsigned char>());
  k_open_x<<<nb, kBlock, 0, s>>>(nx, ny, nz, g.frac_x.as<double>(), g.active.as<unsigned char>(),
                                 g.d_dy.as<double>(), g.d_dz.as<double>(), g.open_x.as<double>());
  k_open_y<<<nb, kBlock, 0, s>>>(nx, ny, nz, g.frac_y.as<double>(), g.active.as<unsigned char>(),
                                 g.d_dx.as<double>(), g.d_dz.as<double>(), g.open_y.as<double>());
  k_open_z<<<nb, kBlock, 0, s>>>(nx, ny, nz, g.frac_z.as<double>(), g.active.as<unsigned char>(),
                                 g.d_dx.as<double>(), g.d_dy.as<double>(), g.open_z.as<double>());
  NFA_CHECK_LAUNCH();
  k_reduced_init<<<blocks_for(n), kBlock, 0, s>>>(n, g.active.as<unsigned char>(),
                                                  g.reduced.as<unsigned char>(), g.root.as<int>());
  NFA_CHECK_LAUNCH();

  std::vector<unsigned char> act(n);
  NFA_HIP(hipMemcpyAsync(act.data(), g.active.p, n, hipMemcpyDeviceToHost, s));
  std::vector<int> target;
  std::vector<double> vf;
  if (psi) {
    DevBuf tbuf;
    NFA_HIP(tbuf.alloc(n * sizeof(int)));
    k_merge_target<<<blocks_for(n), kBlock, 0, s>>>(
        nx, ny, nz, psi, g.vfrac.as<double>(), g.active.as<unsigned char>(), g.open_x.as<double>(),
        g.open_y.as<double>(), g.open_z.as<double>(), g.d_dx.as<double>(), g.d_dy.as<double>(),
        g.d_dz.as<double>(), theta, tbuf.as<int>());
    NFA_CHECK_LAUNCH();
    target.resize(n);
    vf.resize(n);
    NFA_HIP(hipMemcpyAsync(target.data(), tbuf.p, n * sizeof(int), hipMemcpyDeviceToHost, s));
    NFA_HIP(hipMemcpyAsync(vf.data(), g.vfrac.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    NFA_HIP(hipStreamSynchronize(s));
  } else {
    NFA_HIP(hipStreamSynchronize(s));
  }
  long long nact = 0;
  for (long long c = 0; c < n; ++c) nact += act[c];
  g.n_active = nact;

  // resolve merge roots along target chains; a cycle's root is its member
  // with the largest fraction (then the lowest index)
  std::unordered_map<long long, long long> resolved;
  std::vector<long long> small;
  for (long long c = 0; c < (long long)target.size(); ++c)
    if (target[c] >= 0) small.push_back(c);
  for (long long c : small) {
    if (resolved.count(c)) continue;
    std::vector<long long> path;
    std::unordered_map<long long, size_t> pos;
    long long cur = c;
    while (target[cur] >= 0 && !resolved.count(cur) && !pos.count(cur)) {
      pos[cur] = path.size();
      path.push_back(cur);
      cur = target[cur];
    }
    long long r;
    if (resolved.count(cur)) {
      r = resolved[cur];
    } else if (pos.count(cur)) {
      r = -1;
      for (size_t q = pos[cur]; q < path.size(); ++q) {
        const long long m = path[q];
        if (r < 0 || vf[m] > vf[r] || (vf[m] == vf[r] && m < r)) r = m;
      }
    } else {
      r = cur;
    }
    for (long long m : path) resolved[m] = r;
  }
  std::map<long long, std::vector<long long>> groups;
  for (long long c : small) {
    const long long r = resolved[c];
    if (r != c) groups[r].push_back(c);
  }
  std::vector<int> groot, goff, gmem, scell, sroot;
  goff.push_back(0);
  for (auto& kv : groups) {
    std::sort(kv.second.begin(), kv.second.end());
    groot.push_back((int)kv.first);
    for (long long m : kv.second) {
      gmem.push_back((int)m);
      scell.push_back((int)m);
      sroot.push_back((int)kv.first);
    }
    goff.push_back((int)gmem.size());
  }
  g.n_groups = (int)groot.size();
  g.n_slaves = (int)scell.size();
  // rows whose merged-operator row differs from the plain 7-point row of a
  // cell-wise vector: the roots (they carry their slaves' rows) and the
  // unknowns next to a slave (its value is its root's)
  {
    std::unordered_set<long long> slave(scell.begin(), scell.end());
    std::vector<int> fix(groot.begin(), groot.end());
    const long long plane = (long long)nx * ny;
    for (int sc : scell) {
      const long long c = sc;
      const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / plane);
      const long long nbs[6] = {i > 0 ? c - 1 : -1, i < nx - 1 ? c + 1 : -1, j > 0 ? c - nx : -1,
                                j < ny - 1 ? c + nx : -1, k > 0 ? c - plane : -1, k < nz - 1 ? c + plane : -1};
      for (long long nb : nbs)
        if (nb >= 0 && act[nb] && !slave.count(nb)) fix.push_back((int)nb);
    }
    std::sort(fix.begin(), fix.end());
    fix.erase(std::unique(fix.begin(), fix.end()), fix.end());
    g.h_fix = fix;
    g.h_scell = scell;
    g.h_sroot = sroot;
    NFA_HIP(upload_vec(g.fix_rows, fix));
  }
  ++g.body_version;
  g.n_reduced = nact - g.n_slaves;
  NFA_HIP(upload_vec(g.g_root, groot));
  NFA_HIP(upload_vec(g.g_off, goff));
  NFA_HIP(upload_vec(g.g_mem, gmem));
  NFA_HIP(upload_vec(g.s_cell, scell));
  NFA_HIP(upload_vec(g.s_root, sroot));
  if (g.n_slaves > 0) {
    k_reduced_slaves<<<blocks_for(g.n_slaves), kBlock, 0, s>>>(
        g.n_slaves, g.s_cell.as<int>(), g.s_root.as<int>(), g.reduced.as<unsigned char>(),
        g.root.as<int>());
    NFA_CHECK_LAUNCH();
  }
  NFA_HIP(hipStreamSynchronize(s));
  g.has_body = psi != nullptr;
  return NFA_OK;
}

}  // namespace
}  // namespace nfa

using namespace nfa;

extern "C" nfa_status nfa_grid_create(int nx, int ny, int nz, const double* xf, const double* yf,
                                      const double* zf, const int* bc, nfa_grid* out) {
  if (!out) return fail(NFA_ERR_INVALID, "nfa_grid_create: out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return fail(NFA_ERR_INVALID, "nfa_grid_create: sizes must be >= 1");
  if ((long long)(nx + 1) * (ny + 1) * (nz + 1) > 2147483647LL)
    return fail(NFA_ERR_INVALID, "nfa_grid_create: node count exceeds int32 indexing");
  if (!xf || !yf || !zf || !bc) return fail(NFA_ERR_INVALID, "nfa_grid_create: NULL argument");
  const double* fs[3] = {xf, yf, zf};
  const int ns[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < ns[a]; ++i)
      if (!(fs[a][i + 1] > fs[a][i]) || !std::isfinite(fs[a][i]) || !std::isfinite(fs[a][i + 1]))
        return fail(NFA_ERR_INVALID, "nfa_grid_create: face coordinates must be finite and strictly increasing");
  for (int f = 0; f < 6; ++f)
    if (bc[f] != NFA_BC_NEUMANN && bc[f] != NFA_BC_DIRICHLET)
      return fail(NFA_ERR_INVALID, "nfa_grid_create: bc flags must be 0 or 1");
  auto* g = new nfa_grid_s();
  g->nx = nx;
  g->ny = ny;
  g->nz = nz;
  g->n = (long long)nx * ny * nz;
  for (int f = 0; f < 6; ++f) g->bc[f] = bc[f];
  axis_metrics(xf, nx, g->xf, g->dx, g->hx);
  axis_metrics(yf, ny, g->yf, g->dy, g->hy);
  axis_metrics(zf, nz, g->zf, g->dz, g->hz);
  auto bad = [&](hipError_t e) {
    delete g;
    return fail(NFA_ERR_HIP, std::string("nfa_grid_create: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = upload(g->d_dx, g->dx)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_dy, g->dy)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_dz, g->dz)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_hx, g->hx)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_hy, g->hy)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_hz, g->hz)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_gx, normal_den(g->xf))) != hipSuccess) return bad(e);
  if ((e = upload(g->d_gy, normal_den(g->yf))) != hipSuccess) return bad(e);
  if ((e = upload(g->d_gz, normal_den(g->zf))) != hipSuccess) return bad(e);
  if ((e = upload(g->d_xf, g->xf)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_yf, g->yf)) != hipSuccess) return bad(e);
  if ((e = upload(g->d_zf, g->zf)) != hipSuccess) return bad(e);
  const long long n = g->n;
  if ((e = g->frac_x.alloc(g->nfx() * 8)) != hipSuccess) return bad(e);
  if ((e = g->frac_y.alloc(g->nfy() * 8)) != hipSuccess) return bad(e);
  if ((e = g->frac_z.alloc(g->nfz() * 8)) != hipSuccess) return bad(e);
  if ((e = g->open_x.alloc(g->nfx() * 8)) != hipSuccess) return bad(e);
  if ((e = g->open_y.alloc(g->nfy() * 8)) != hipSuccess) return bad(e);
  if ((e = g->open_z.alloc(g->nfz() * 8)) != hipSuccess) return bad(e);
  if ((e = g->vfrac.alloc(n * 8)) != hipSuccess) return bad(e);
  if ((e = g->active.alloc(n)) != hipSuccess) return bad(e);
  if ((e = g->reduced.alloc(n)) != hipSuccess) return bad(e);
  if ((e = g->root.alloc(n * 4)) != hipSuccess) return bad(e);
  nfa_status st = compute_body(*g, nullptr, 0.0, 1, nullptr);
  if (st != NFA_OK) {
    delete g;
    return st;
  }
  *out = g;
  return NFA_OK;
}

extern "C" nfa_status nfa_grid_set_body(nfa_grid g, const double* psi, double theta, int samples,
                                        nfa_stream s) {
  if (!g) return fail(NFA_ERR_INVALID, "nfa_grid_set_body: NULL grid");
  if (!(theta >= 0.0 && theta < 1.0)) return fail(NFA_ERR_INVALID, "nfa_grid_set_body: theta must be in [0,1)");
  if (samples < 1 || samples > 64) return fail(NFA_ERR_INVALID, "nfa_grid_set_body: samples must be in [1,64]");
  return compute_body(*g, psi, theta, samples, S(s));
}

extern "C" nfa_status nfa_grid_get_info(nfa_grid g, nfa_grid_info* info) {
  if (!g || !info) return fail(NFA_ERR_INVALID, "nfa_grid_get_info: NULL argument");
  info->nx = g->nx;
  info->ny = g->ny;
  info->nz = g->nz;
  info->cells = g->n;
  info->active = g->n_active;
  info->reduced = g->n_reduced;
  info->groups = g->n_groups;
  info->slaves = g->n_slaves;
  info->all_neumann = g->all_neumann() ? 1 : 0;
  return NFA_OK;
}

extern "C" nfa_status nfa_grid_export(nfa_grid g, int what, void* dst, nfa_stream s) {
  if (!g || !dst) return fail(NFA_ERR_INVALID, "nfa_grid_export: NULL argument");
  const DevBuf* b = nullptr;
  switch (what) {
    case NFA_EXPORT_FRAC_X: b = &g->frac_x; break;
    case NFA_EXPORT_FRAC_Y: b = &g->frac_y; break;
    case NFA_EXPORT_FRAC_Z: b = &g->frac_z; break;
    case NFA_EXPORT_VFRAC: b = &g->vfrac; break;
    case NFA_EXPORT_OPEN_X: b = &g->open_x; break;
    case NFA_EXPORT_OPEN_Y: b = &g->open_y; break;
    case NFA_EXPORT_OPEN_Z: b = &g->open_z; break;
    case NFA_EXPORT_ACTIVE: b = &g->active; break;
    case NFA_EXPORT_ROOT: b = &g->root; break;
    case NFA_EXPORT_REDUCED: b = &g->reduced; break;
    default: return fail(NFA_ERR_INVALID, "nfa_grid_export: unknown item");
  }
  NFA_HIP(hipMemcpyAsync(dst, b->p, b->bytes, hipMemcpyDeviceToDevice, S(s)));
  return NFA_OK;
}

extern "C" void nfa_grid_destroy(nfa_grid g) { delete g; }
