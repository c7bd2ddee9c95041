// Once-per-mesh work (H0): node -> element lists, the node graph, the CSR
// pattern of all element-coupled dof pairs and the per-element table of
// neighbour positions used by the assembly.  The paper forms triplets per
// element and lets sparse() sum duplicates inside every iteration (Fig. 2);
// here the pattern is built once and every Newton iteration writes values
// into it.  All lists are sorted, so the result is deterministic although
// the fill uses atomic cursors.
#include <hipcub/hipcub.hpp>

#include "lgdm_internal.h"

namespace lgdm {

namespace {

constexpr int MAX_ELEM_PER_NODE = 16;   // per node, any element type
constexpr int MAX_CAND = 160;          // element nodes gathered per node: elements x nodes per element

__global__ void count_n2e_kernel(int64_t n, const int32_t* __restrict__ conn,
                                 int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[conn[i]], 1);
}

__global__ void fill_n2e_kernel(int64_t n, int nen, const int32_t* __restrict__ conn,
                                const int32_t* __restrict__ ptr, int32_t* __restrict__ cursor,
                                int32_t* __restrict__ n2e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t node = conn[i];
  const int32_t e = (int32_t)(i / nen), la = (int32_t)(i % nen);
  const int32_t slot = atomicAdd(&cursor[node], 1);
  n2e[ptr[node] + slot] = (e << N2E_SHIFT) | la;
}

__device__ void isort(int32_t* v, int n) {
  for (int i = 1; i < n; ++i) {
    const int32_t t = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > t) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = t;
  }
}

__global__ void sort_n2e_kernel(int64_t n_nodes, const int32_t* __restrict__ ptr,
                                int32_t* __restrict__ n2e, int32_t* __restrict__ stats) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_nodes) return;
  const int s = ptr[a], n = ptr[a + 1] - s;
  atomicMax(&stats[0], n);
  if (n > MAX_ELEM_PER_NODE) return;
  int32_t v[MAX_ELEM_PER_NODE];
  for (int i = 0; i < n; ++i) v[i] = n2e[s + i];
  isort(v, n);
  for (int i = 0; i < n; ++i) n2e[s + i] = v[i];
}

// neighbour set of node a = all nodes of its elements, sorted and unique.
// pass 0 counts, pass 1 writes.
__global__ void nbr_kernel(int64_t n_nodes, int nen, const int32_t* __restrict__ conn,
                           const int32_t* __restrict__ n2e_ptr, const int32_t* __restrict__ n2e,
                           int32_t* __restrict__ cnt, const int32_t* __restrict__ nbr_ptr,
                           int32_t* __restrict__ nbr, int32_t* __restrict__ dpos,
                           int32_t* __restrict__ stats, int pass) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_nodes) return;
  const int s = n2e_ptr[a], ne = n2e_ptr[a + 1] - s;
  if (ne > MAX_ELEM_PER_NODE) return;
  if (ne * nen > MAX_CAND) {
    if (pass == 0) atomicMax(&stats[4], ne * nen);
    return;
  }
  int32_t cand[MAX_CAND];
  int nc = 0;
  for (int i = 0; i < ne; ++i) {
    const int64_t e = n2e[s + i] >> N2E_SHIFT;
    for (int b = 0; b < nen; ++b) cand[nc++] = conn[e * nen + b];
  }
  isort(cand, nc);
  int nu = 0;
  for (int i = 0; i < nc; ++i)
    if (i == 0 || cand[i] != cand[i - 1]) cand[nu++] = cand[i];
  if (pass == 0) {
    cnt[a] = nu;
    atomicMax(&stats[1], nu);
    if (ne == 0) atomicAdd(&stats[2], 1);
  } else {
    const int o = nbr_ptr[a];
    for (int i = 0; i < nu; ++i) {
      nbr[o + i] = cand[i];
      if (cand[i] == a) dpos[a] = i;
    }
  }
}

// dof CSR: rows of node a are a*nd + r; each row lists, for every neighbour
// in ascending order, its nd columns
__global__ void csr_kernel(int64_t n_nodes, int nd, const int32_t* __restrict__ nbr_ptr,
                           const int32_t* __restrict__ nbr, int32_t* __restrict__ row_ptr,
                           int32_t* __restrict__ col_idx) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_nodes) return;
  const int64_t p0 = nbr_ptr[a];
  const int nnb = nbr_ptr[a + 1] - (int)p0;
  const int64_t base = p0 * nd * nd;
  for (int r = 0; r < nd; ++r) {
    const int64_t rs = base + (int64_t)r * nnb * nd;
    row_ptr[a * nd + r] = (int32_t)rs;
    for (int p = 0; p < nnb; ++p) {
      const int32_t b = nbr[p0 + p];
      for (int c = 0; c < nd; ++c) col_idx[rs + (int64_t)p * nd + c] = b * nd + c;
    }
  }
  if (a == n_nodes - 1) row_ptr[n_nodes * nd] = (int32_t)(nbr_ptr[n_nodes] * (int64_t)nd * nd);
}

// position of node b within node a's neighbour list, for every (e, a, b)
__global__ void pos_kernel(int64_t n, int nen, const int32_t* __restrict__ conn,
                           const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                           uint8_t* __restrict__ pos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t e = t / (nen * nen);
  const int la = (int)((t / nen) % nen), lb = (int)(t % nen);
  const int32_t a = conn[e * nen + la], b = conn[e * nen + lb];
  int lo = nbr_ptr[a], hi = nbr_ptr[a + 1] - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nbr[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  pos[t] = (uint8_t)(lo - nbr_ptr[a]);
}

__global__ void check_conn_kernel(int64_t n, int64_t n_nodes, const int32_t* __restrict__ conn,
                                  int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (conn[i] < 0 || conn[i] >= n_nodes)) atomicAdd(bad, 1);
}

inline int64_t blocks(int64_t n, int bs) { return (n + bs - 1) / bs; }

}  // namespace

// Builds everything the assembly needs from c->conn.  status receives an
// lgdm_status (INVALID_ARG for meshes the kernels do not handle).
hipError_t build_pattern(lgdm_ctx* c, std::string& msg, int& status) {
  status = LGDM_OK;
  const int nen = c->nen, nd = c->nd;
  const int64_t nconn = c->n_elems * nen;
  hipStream_t st = c->stream;
  hipError_t e;
  int32_t* stats = (int32_t*)dalloc(c, 8 * sizeof(int32_t));
  int32_t* cnt = (int32_t*)dalloc(c, (c->n_nodes + 1) * sizeof(int32_t));
  int32_t* cursor = (int32_t*)dalloc(c, (c->n_nodes + 1) * sizeof(int32_t));
  c->n2e_ptr = (int32_t*)dalloc(c, (c->n_nodes + 1) * sizeof(int32_t));
  c->nbr_ptr = (int32_t*)dalloc(c, (c->n_nodes + 1) * sizeof(int32_t));
  c->dpos = (int32_t*)dalloc(c, c->n_nodes * sizeof(int32_t));
  c->n2e = (int32_t*)dalloc(c, (nconn > 0 ? nconn : 1) * sizeof(int32_t));
  if (!stats || !cnt || !cursor || !c->n2e_ptr || !c->nbr_ptr || !c->dpos || !c->n2e) {
    status = LGDM_ERR_OOM;
    msg = "device allocation failed while building the pattern";
    return hipSuccess;
  }
  int32_t h_stats[8] = {0};
  if ((e = hipMemsetAsync(stats, 0, 8 * sizeof(int32_t), st)) != hipSuccess) return e;
  check_conn_kernel<<<blocks(nconn, 256), 256, 0, st>>>(nconn, c->n_nodes, c->conn, stats + 3);
  if ((e = hipMemcpyAsync(h_stats, stats, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (h_stats[3] != 0) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "connectivity holds node ids outside [0, n_nodes)";
    return hipSuccess;
  }
  // node -> element lists
  if ((e = hipMemsetAsync(cnt, 0, (c->n_nodes + 1) * sizeof(int32_t), st)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cursor, 0, (c->n_nodes + 1) * sizeof(int32_t), st)) != hipSuccess) return e;
  count_n2e_kernel<<<blocks(nconn, 256), 256, 0, st>>>(nconn, c->conn, cnt);
  size_t tmp_bytes = 0;
  if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, c->n2e_ptr,
                                            (int)(c->n_nodes + 1), st)) != hipSuccess) return e;
  void* tmp = dalloc(c, tmp_bytes > 0 ? tmp_bytes : 1);
  if (!tmp) {
    status = LGDM_ERR_OOM;
    msg = "device allocation failed while building the pattern";
    return hipSuccess;
  }
  if ((e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, c->n2e_ptr, (int)(c->n_nodes + 1),
                                            st)) != hipSuccess) return e;
  fill_n2e_kernel<<<blocks(nconn, 256), 256, 0, st>>>(nconn, nen, c->conn, c->n2e_ptr, cursor, c->n2e);
  sort_n2e_kernel<<<blocks(c->n_nodes, 256), 256, 0, st>>>(c->n_nodes, c->n2e_ptr, c->n2e, stats);
  // node graph
  nbr_kernel<<<blocks(c->n_nodes, 128), 128, 0, st>>>(c->n_nodes, nen, c->conn, c->n2e_ptr, c->n2e,
                                                      cnt, nullptr, nullptr, nullptr, stats, 0);
  if ((e = hipMemsetAsync(cnt + c->n_nodes, 0, sizeof(int32_t), st)) != hipSuccess) return e;
  if ((e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, c->nbr_ptr, (int)(c->n_nodes + 1),
                                            st)) != hipSuccess) return e;
  int32_t npairs = 0;
  if ((e = hipMemcpyAsync(&npairs, c->nbr_ptr + c->n_nodes, sizeof(int32_t), hipMemcpyDeviceToHost,
                          st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(h_stats, stats, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  dfree(c, tmp);
  c->max_elem_per_node = h_stats[0];
  c->max_nbr = h_stats[1];
  const int lanes = nen * nen;
  if (h_stats[0] > MAX_ELEM_PER_NODE) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "a node is shared by more than 16 elements";
    return hipSuccess;
  }
  if (h_stats[4] > 0) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "a node's elements list more node entries than the pattern builder handles";
    return hipSuccess;
  }
  if (h_stats[1] > lanes || h_stats[1] > 255) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "a node has more neighbours than the assembly kernel handles (" +
          std::to_string(lanes) + " for this element type)";
    return hipSuccess;
  }
  if (h_stats[2] > 0) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "mesh has nodes that belong to no element";
    return hipSuccess;
  }
  c->npairs = npairs;
  const int64_t nnz = (int64_t)npairs * nd * nd;
  if (nnz >= (int64_t)1 << 31) {
    status = LGDM_ERR_INVALID_ARG;
    msg = "nnz >= 2^31: int32 CSR indices cannot address this mesh";
    return hipSuccess;
  }
  c->nnz = nnz;
  c->nbr = (int32_t*)dalloc(c, (npairs > 0 ? npairs : 1) * sizeof(int32_t));
  c->row_ptr = (int32_t*)dalloc(c, (c->ndof + 1) * sizeof(int32_t));
  c->col_idx = (int32_t*)dalloc(c, (nnz > 0 ? nnz : 1) * sizeof(int32_t));
  c->pos = (uint8_t*)dalloc(c, (c->n_elems * nen * nen > 0 ? c->n_elems * nen * nen : 1));
  if (!c->nbr || !c->row_ptr || !c->col_idx || !c->pos) {
    status = LGDM_ERR_OOM;
    msg = "device allocation failed while building the pattern";
    return hipSuccess;
  }
  nbr_kernel<<<blocks(c->n_nodes, 128), 128, 0, st>>>(c->n_nodes, nen, c->conn, c->n2e_ptr, c->n2e,
                                                      cnt, c->nbr_ptr, c->nbr, c->dpos, stats, 1);
  csr_kernel<<<blocks(c->n_nodes, 128), 128, 0, st>>>(c->n_nodes, nd, c->nbr_ptr, c->nbr, c->row_ptr,
                                                      c->col_idx);
  const int64_t npos = c->n_elems * nen * nen;
  pos_kernel<<<blocks(npos, 256), 256, 0, st>>>(npos, nen, c->conn, c->nbr_ptr, c->nbr, c->pos);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  dfree(c, cnt);
  dfree(c, cursor);
  dfree(c, stats);
  return hipSuccess;
}

}  // namespace lgdm
