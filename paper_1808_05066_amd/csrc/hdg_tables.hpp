// Reference-element tables and element geometry, built on the host.
//
// The discretization spaces are the paper's (P_k on simplices, the tensor space
// Q_k on quads / hexes); nodes and quadrature follow the library's documented
// reading: Gauss-Lobatto tensor nodes or equispaced simplex nodes, Gauss-Legendre
// rules with p+2 points per direction, collapsed (Duffy) on simplices.
//
// Everything here is computed from first principles: Newton iteration on the
// Legendre recurrence for Gauss and Gauss-Lobatto points, barycentric Lagrange
// products for the tensor bases, Silvester's product formula for the
// equispaced simplex bases, Nanson's relation for face normals.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hdg {

enum EType { TRI = 0, QUAD = 1, TET = 2, HEX = 3 };

struct RefTables {
  int etype = 0, p = 0, dim = 0, m = 0, Np = 0, nf = 0, Nfp = 0, Nq = 0, Nfq = 0, nv = 0;
  std::vector<int> mi;        // [Np][dim] node multi-indices
  std::vector<double> nodes;  // [Np][dim] reference node coordinates
  std::vector<double> xq;     // [Nq][dim]
  std::vector<double> wq;     // [Nq]
  std::vector<double> phi;    // [Nq][Np]
  std::vector<double> dphi;   // [dim][Nq][Np]
  std::vector<int> fnodes;    // [nf][Nfp]
  std::vector<double> fxi;    // [nf][Nfq][dim]
  std::vector<double> fw;     // [nf][Nfq] rule weight times reference face area factor
  std::vector<double> fnref;  // [nf][dim] unit outward reference normal
  std::vector<double> fphi;   // [nf][Nfq][Nfp] face-node basis at face points
  std::vector<double> vref;   // [nv][dim] reference vertices
};

// Build tables; returns an empty string on success or an error message.
std::string build_ref_tables(int etype, int p, RefTables &t);

// Basis values [N][Np] and reference gradients [dim][N][Np] at points x [N][dim].
void eval_basis(const RefTables &t, const double *x, int N, double *val, double *grad);

// Vertex shape functions [nv] and reference gradients [nv][dim] at one point.
void vertex_shape(int etype, int dim, const double *xi, double *N, double *dN);

// 1D rules.
void gauss_legendre(int n, double *x, double *w);
void gll_points(int p, double *x);

}  // namespace hdg
