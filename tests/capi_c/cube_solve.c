/*
 * cube_solve.c - drives the solver through its C ABI alone (include/vem.h and
 * the HIP runtime's C API; no Python, no PyTorch).
 *
 * Builds the structured n^3 hexahedral mesh of the unit cube (the same
 * numbering as the Python input generator: vertex (i,j,k) -> i + (n+1)(j +
 * (n+1)k); x-, then y-, then z-normal faces, each normal along +axis; cell
 * faces in the order -x, +x, -y, +y, -z, +z), discretises the lowest-order
 * element, sets nu = 1/K per cell from a file, evaluates the load
 * f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the library's quadrature points
 * (p_D = 0), solves with the chosen block preconditioner and writes u then p
 * (FP64, native byte order) to a file.
 *
 * usage: cube_solve n nu_file out_file [schur|reg [batch B]]
 *        prints one line: n_u n_p iterations relres status
 *        With "batch B", nu_file holds B fields (B n^3 doubles): they are set with
 *        vem_set_coefficient_batch and solved with vem_solve_batch (one load for all), the B
 *        solutions are written one after another, and one line per field is printed.
 *        cube_solve --mesh n out_file
 *        writes the mesh arrays only (no GPU call): nv, nf, nc (int64), xyz,
 *        face_ptr, face_vtx, cell_ptr, cell_face (int32), cell_face_sign (int8)
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vem.h"

static vem_handle g_h = NULL;

#define CHECK_HIP(call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      fprintf(stderr, "%s:%d: %s failed: %s\n", __FILE__, __LINE__, #call,                \
              hipGetErrorString(e_));                                                      \
      exit(2);                                                                             \
    }                                                                                      \
  } while (0)

#define CHECK_VEM(call)                                                                    \
  do {                                                                                     \
    vem_status s_ = (call);                                                                \
    if (s_ < 0) {                                                                          \
      fprintf(stderr, "%s:%d: %s failed: %s (%s)\n", __FILE__, __LINE__, #call,           \
              vem_status_string(s_), g_h ? vem_last_error(g_h) : "");                      \
      exit(3);                                                                             \
    }                                                                                      \
  } while (0)

static void* xmalloc(size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of host memory\n");
    exit(4);
  }
  return p;
}

typedef struct {
  int64_t nv, nf, nc;
  double* xyz;
  int32_t *face_ptr, *face_vtx, *cell_ptr, *cell_face;
  int8_t* sign;
} cube_mesh;

static cube_mesh make_cube(int n) {
  const int64_t v = n + 1;
  cube_mesh m;
  m.nv = v * v * v;
  const int64_t nfx = v * n * n, nfy = n * v * n, nfz = n * n * v;
  m.nf = nfx + nfy + nfz;
  m.nc = (int64_t)n * n * n;
  m.xyz = xmalloc(sizeof(double) * 3 * m.nv);
  m.face_ptr = xmalloc(sizeof(int32_t) * (m.nf + 1));
  m.face_vtx = xmalloc(sizeof(int32_t) * 4 * m.nf);
  m.cell_ptr = xmalloc(sizeof(int32_t) * (m.nc + 1));
  m.cell_face = xmalloc(sizeof(int32_t) * 6 * m.nc);
  m.sign = xmalloc(sizeof(int8_t) * 6 * m.nc);
#define VID(i, j, k) ((int32_t)((i) + v * ((j) + v * (k))))
  for (int64_t k = 0; k < v; ++k)
    for (int64_t j = 0; j < v; ++j)
      for (int64_t i = 0; i < v; ++i) {
        const int32_t id = VID(i, j, k);
        m.xyz[3 * id + 0] = (double)i / n;
        m.xyz[3 * id + 1] = (double)j / n;
        m.xyz[3 * id + 2] = (double)k / n;
      }
  for (int64_t f = 0; f <= m.nf; ++f) m.face_ptr[f] = (int32_t)(4 * f);
  /* x-normal faces: counter-clockwise about +x */
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < v; ++i) {
        int32_t* q = m.face_vtx + 4 * (i + v * (j + n * k));
        q[0] = VID(i, j, k), q[1] = VID(i, j + 1, k), q[2] = VID(i, j + 1, k + 1), q[3] = VID(i, j, k + 1);
      }
  /* y-normal faces: counter-clockwise about +y */
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < v; ++j)
      for (int64_t i = 0; i < n; ++i) {
        int32_t* q = m.face_vtx + 4 * (nfx + i + n * (j + v * k));
        q[0] = VID(i, j, k), q[1] = VID(i, j, k + 1), q[2] = VID(i + 1, j, k + 1), q[3] = VID(i + 1, j, k);
      }
  /* z-normal faces: counter-clockwise about +z */
  for (int64_t k = 0; k < v; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        int32_t* q = m.face_vtx + 4 * (nfx + nfy + i + n * (j + n * k));
        q[0] = VID(i, j, k), q[1] = VID(i + 1, j, k), q[2] = VID(i + 1, j + 1, k), q[3] = VID(i, j + 1, k);
      }
#undef VID
  for (int64_t c = 0; c <= m.nc; ++c) m.cell_ptr[c] = (int32_t)(6 * c);
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        const int64_t c = i + n * (j + n * k);
        int32_t* cf = m.cell_face + 6 * c;
        cf[0] = (int32_t)(i + v * (j + n * k));
        cf[1] = (int32_t)(i + 1 + v * (j + n * k));
        cf[2] = (int32_t)(nfx + i + n * (j + v * k));
        cf[3] = (int32_t)(nfx + i + n * (j + 1 + v * k));
        cf[4] = (int32_t)(nfx + nfy + i + n * (j + n * k));
        cf[5] = (int32_t)(nfx + nfy + i + n * (j + n * (k + 1)));
        for (int a = 0; a < 6; ++a) m.sign[6 * c + a] = (int8_t)(a % 2 ? 1 : -1);
      }
  return m;
}

static void free_cube(cube_mesh* m) {
  free(m->xyz), free(m->face_ptr), free(m->face_vtx), free(m->cell_ptr), free(m->cell_face), free(m->sign);
}

static int dump_mesh(int n, const char* path) {
  cube_mesh m = make_cube(n);
  FILE* fo = fopen(path, "wb");
  if (!fo) return 1;
  const int64_t head[3] = {m.nv, m.nf, m.nc};
  int ok = fwrite(head, sizeof(int64_t), 3, fo) == 3;
  ok = ok && fwrite(m.xyz, sizeof(double), (size_t)(3 * m.nv), fo) == (size_t)(3 * m.nv);
  ok = ok && fwrite(m.face_ptr, sizeof(int32_t), (size_t)(m.nf + 1), fo) == (size_t)(m.nf + 1);
  ok = ok && fwrite(m.face_vtx, sizeof(int32_t), (size_t)(4 * m.nf), fo) == (size_t)(4 * m.nf);
  ok = ok && fwrite(m.cell_ptr, sizeof(int32_t), (size_t)(m.nc + 1), fo) == (size_t)(m.nc + 1);
  ok = ok && fwrite(m.cell_face, sizeof(int32_t), (size_t)(6 * m.nc), fo) == (size_t)(6 * m.nc);
  ok = ok && fwrite(m.sign, sizeof(int8_t), (size_t)(6 * m.nc), fo) == (size_t)(6 * m.nc);
  fclose(fo);
  free_cube(&m);
  return ok ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc == 4 && strcmp(argv[1], "--mesh") == 0) {
    const int n = atoi(argv[2]);
    if (n < 1 || n > 512) {
      fprintf(stderr, "n must be in 1..512\n");
      return 1;
    }
    return dump_mesh(n, argv[3]);
  }
  if (argc < 4) {
    fprintf(stderr, "usage: %s n nu_file out_file [schur|reg]\n", argv[0]);
    return 1;
  }
  const int n = atoi(argv[1]);
  if (n < 1 || n > 512) {
    fprintf(stderr, "n must be in 1..512\n");
    return 1;
  }
  const int reg = argc > 4 && strcmp(argv[4], "reg") == 0;
  const int nb = (argc > 6 && strcmp(argv[5], "batch") == 0) ? atoi(argv[6]) : 0;
  if (argc > 5 && (nb < 1 || nb > 64)) {
    fprintf(stderr, "batch B: B must be in 1..64\n");
    return 1;
  }
  cube_mesh m = make_cube(n);

  /* nu per cell, n^3 doubles per field */
  const int64_t nfield = nb > 0 ? nb : 1;
  double* nu = xmalloc(sizeof(double) * m.nc * nfield);
  FILE* fin = fopen(argv[2], "rb");
  if (!fin || fread(nu, sizeof(double), (size_t)(m.nc * nfield), fin) != (size_t)(m.nc * nfield)) {
    fprintf(stderr, "cannot read %lld coefficients from %s\n", (long long)(m.nc * nfield), argv[2]);
    return 1;
  }
  fclose(fin);

  CHECK_VEM(vem_create(&g_h, NULL));
  CHECK_VEM(vem_set_mesh(g_h, m.nv, m.xyz, m.nf, m.face_ptr, m.face_vtx, m.nc, m.cell_ptr, m.cell_face, m.sign,
                         VEM_MEM_HOST));
  CHECK_VEM(vem_discretize(g_h, VEM_LO, 0, 3));
  vem_sizes sz;
  CHECK_VEM(vem_get_sizes(g_h, &sz));
  CHECK_VEM(vem_set_coefficient(g_h, nu));

  /* the load at the library's volume quadrature points (structure of arrays) */
  const int64_t nq = sz.n_qp_cell;
  double *qc_d = NULL, *f_d = NULL;
  CHECK_HIP(hipMalloc((void**)&qc_d, sizeof(double) * 3 * nq));
  CHECK_HIP(hipMalloc((void**)&f_d, sizeof(double) * nq));
  CHECK_VEM(vem_get_quadrature(g_h, qc_d, NULL));
  double* qc = xmalloc(sizeof(double) * 3 * nq);
  double* f = xmalloc(sizeof(double) * nq);
  CHECK_HIP(hipMemcpy(qc, qc_d, sizeof(double) * 3 * nq, hipMemcpyDeviceToHost));
  const double pi = 3.14159265358979323846;
  for (int64_t q = 0; q < nq; ++q)
    f[q] = 3.0 * pi * pi * (sin(pi * qc[q]) * sin(pi * qc[nq + q]) * sin(pi * qc[2 * nq + q]));
  CHECK_HIP(hipMemcpy(f_d, f, sizeof(double) * nq, hipMemcpyHostToDevice));
  CHECK_VEM(vem_set_rhs(g_h, f_d, NULL));

  vem_solve_opts o;
  vem_solve_opts_default(&o);
  o.precond = reg ? VEM_PREC_REG : VEM_PREC_SCHUR;
  o.tol = 1e-12;
  o.inner_tol = reg ? 1e-1 : 1e-10;
  o.maxit = 5000;
  double *u_d = NULL, *p_d = NULL;
  CHECK_HIP(hipMalloc((void**)&u_d, sizeof(double) * sz.n_u * nfield));
  CHECK_HIP(hipMalloc((void**)&p_d, sizeof(double) * sz.n_p * nfield));
  vem_solve_info info[64];
  vem_status st;
  if (nb > 0) {
    /* the fields in host memory; the library copies them in */
    CHECK_VEM(vem_set_coefficient_batch(g_h, nb, nu));
    st = vem_solve_batch(g_h, &o, nb, u_d, p_d, info);
  } else {
    st = vem_solve(g_h, &o, u_d, p_d, info);
  }
  CHECK_VEM(st);

  const int64_t nx = sz.n_u + sz.n_p;
  double* x = xmalloc(sizeof(double) * nx * nfield);
  for (int64_t b = 0; b < nfield; ++b) {
    CHECK_HIP(hipMemcpy(x + b * nx, u_d + b * sz.n_u, sizeof(double) * sz.n_u, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(x + b * nx + sz.n_u, p_d + b * sz.n_p, sizeof(double) * sz.n_p, hipMemcpyDeviceToHost));
  }
  FILE* fout = fopen(argv[3], "wb");
  if (!fout || fwrite(x, sizeof(double), (size_t)(nx * nfield), fout) != (size_t)(nx * nfield)) {
    fprintf(stderr, "cannot write %s\n", argv[3]);
    return 1;
  }
  fclose(fout);
  for (int64_t b = 0; b < nfield; ++b)
    printf("%lld %lld %d %.6e %d\n", (long long)sz.n_u, (long long)sz.n_p, info[b].iterations, info[b].relres,
           info[b].status);

  CHECK_HIP(hipFree(qc_d));
  CHECK_HIP(hipFree(f_d));
  CHECK_HIP(hipFree(u_d));
  CHECK_HIP(hipFree(p_d));
  CHECK_VEM(vem_destroy(g_h));
  free(qc), free(f), free(x), free(nu);
  free_cube(&m);
  return 0;
}
