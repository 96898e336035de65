// The divergence and gradient kernels' phases run on the CPU: each phase for
// every thread index of the work-group in turn, element by element, with the
// LDS buffers on the heap, so that an address sanitizer build checks every
// shared and global access of the kernels' index arithmetic.  Either the
// projection's pair (velocity degree P, pressure degree P-1) or the equal-order
// pair (scalar degree P, the divergence also in its nodal form, M^-1 times a
// nodal factor, and the gradient with that factor).  Reads the mesh and the
// fields from a binary file and writes the divergence and the gradient.
//
//   projection_phases P nx ny nz bcx bcy bcz with_vb equal in.bin out.bin
//   in.bin:  h_x[nx] h_y[ny] h_z[nz] v0 v1 v2 [vb0 vb1 vb2] psi [fac]  (float64)
//   out.bin: div[Nq] [div_nodal[N]] g0[N] g1[N] g2[N]   (Nq = N when equal, else Np)
#include "projection.hip"
#include "gll_host.cpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>

namespace dg {
void set_error(const std::string &) {}
const GllTables &gll_cached(int P)
{
    static std::map<int, std::unique_ptr<GllTables>> cache;
    auto it = cache.find(P);
    if (it == cache.end()) it = cache.emplace(P, std::make_unique<GllTables>(make_gll(P))).first;
    return *it->second;
}
namespace {
template <int P>
void run_elements(const ProjArgs &A, int nel)
{
    constexpr int Q = P - 1;
    using D = DivShape<P, Q>;
    using G = GradShape<P, Q>;
    for (int el = 0; el < nel; ++el) {
        std::vector<double> tw(P + 1), a(D::BUF_A), b(D::BUF_B);
        for (int t = 0; t < D::NT; ++t) proj_weights<P>(A, t, D::NT, tw.data());
        for (int t = 0; t < D::NT; ++t) div_load<P, Q>(A, el, t, D::NT, tw.data(), a.data());
        for (int t = 0; t < D::NT; ++t) div_pass1<P, Q>(A.t, t, a.data(), b.data());
        for (int t = 0; t < D::NT; ++t) div_pass2<P, Q>(A.t, t, b.data(), a.data());
        for (int t = 0; t < D::NT; ++t) div_pass3<P, Q>(A, A.t, el, t, a.data(), b.data());
        for (int t = 0; t < D::NT; ++t) div_store<P, Q>(A, el, t, D::NT, b.data());
        std::vector<double> q(G::m3), qn(6 * G::m * G::m), ga(G::BUF_A), gb(G::BUF_B);
        for (int t = 0; t < G::NT; ++t) grad_load<P, Q>(A, el, t, G::NT, q.data(), qn.data());
        for (int t = 0; t < G::NT; ++t) grad_pass1<P, Q>(A, A.t, el, t, q.data(), qn.data(), ga.data());
        for (int t = 0; t < G::NT; ++t) grad_pass2<P, Q>(A.t, t, ga.data(), gb.data());
        for (int t = 0; t < G::NT; ++t) grad_pass3<P, Q>(A.t, t, gb.data(), ga.data());
        for (int t = 0; t < G::NT; ++t) grad_store<P, Q>(A, el, t, G::NT, tw.data(), ga.data());
    }
}

template <int P>
void run_elements_equal(const ProjArgs &A, int nel, double *out2)
{
    using S = EqShape<P>;
    for (int el = 0; el < nel; ++el) {
        // the weak divergence into out, its nodal form (M^-1, times fac) into
        // out2
        for (int nodal = 0; nodal < 2; ++nodal) {
            ProjArgs B = A;
            B.nodal = nodal;
            if (nodal) B.out = out2;
            std::vector<double> tv(3 * S::n3), fv(6 * S::n2), tw(S::n);
            for (int t = 0; t < S::NT; ++t) eqdiv_load<P>(B, el, t, tv.data(), fv.data(), tw.data());
            for (int t = 0; t < S::NT; ++t) eqdiv_lines<P>(B, B.t, el, t, tv.data(), fv.data(), tw.data());
            for (int t = 0; t < S::NT; ++t) eqdiv_store<P>(B, el, t, tv.data(), tw.data());
        }
        std::vector<double> q(S::n3), qn(6 * S::n2), R(3 * S::n3);
        for (int t = 0; t < S::NT; ++t) eqgrad_load<P>(A, el, t, q.data(), qn.data());
        for (int t = 0; t < S::NT; ++t) eqgrad_lines<P>(A, A.t, el, t, q.data(), qn.data(), R.data());
        for (int t = 0; t < S::NT; ++t) eqgrad_store<P>(A, el, t, R.data());
    }
}
}  // namespace
}  // namespace dg

int main(int argc, char **argv)
{
    if (argc != 12) {
        fprintf(stderr, "usage: %s P nx ny nz bcx bcy bcz with_vb equal in.bin out.bin\n", argv[0]);
        return 2;
    }
    const int P = atoi(argv[1]);
    const int n[3] = {atoi(argv[2]), atoi(argv[3]), atoi(argv[4])};
    const int bc[3] = {atoi(argv[5]), atoi(argv[6]), atoi(argv[7])};
    const int with_vb = atoi(argv[8]), equal = atoi(argv[9]);
    const int nel = n[0] * n[1] * n[2];
    const size_t N = (size_t)nel * (P + 1) * (P + 1) * (P + 1);
    const size_t Np = equal ? N : (size_t)nel * P * P * P;
    FILE *f = fopen(argv[10], "rb");
    if (!f) return 3;
    auto read = [&](size_t k) {
        std::vector<double> v(k);
        if (fread(v.data(), sizeof(double), k, f) != k) exit(3);
        return v;
    };
    const std::vector<double> h[3] = {read(n[0]), read(n[1]), read(n[2])};
    std::vector<double> v[3], vb[3];
    for (int d = 0; d < 3; ++d) v[d] = read(N);
    if (with_vb)
        for (int d = 0; d < 3; ++d) vb[d] = read(N);
    const std::vector<double> psi = read(Np);
    const std::vector<double> fac = equal ? read(N) : std::vector<double>();
    fclose(f);
    std::vector<double> div(Np, -999.0), div2(equal ? N : 0, -999.0), g[3];
    dg::ProjArgs A{};
    A.t = dg::make_tables(P, equal ? P : P - 1);
    for (int d = 0; d < 3; ++d) {
        g[d].assign(N, -999.0);
        A.n[d] = n[d];
        A.bc[d] = bc[d];
        A.v[d] = v[d].data();
        A.vb[d] = with_vb ? vb[d].data() : nullptr;
        A.g[d] = g[d].data();
        A.h[d] = h[d].data();
    }
    A.psi = psi.data();
    A.out = div.data();
    A.scale = 1.0;
    A.fac = equal ? fac.data() : nullptr;
    if (equal) {
        switch (P) {
            case 3: dg::run_elements_equal<3>(A, nel, div2.data()); break;
            case 4: dg::run_elements_equal<4>(A, nel, div2.data()); break;
            case 5: dg::run_elements_equal<5>(A, nel, div2.data()); break;
            case 6: dg::run_elements_equal<6>(A, nel, div2.data()); break;
            case 7: dg::run_elements_equal<7>(A, nel, div2.data()); break;
            case 8: dg::run_elements_equal<8>(A, nel, div2.data()); break;
            default: return 4;
        }
    } else {
        switch (P) {
            case 4: dg::run_elements<4>(A, nel); break;
            case 5: dg::run_elements<5>(A, nel); break;
            case 6: dg::run_elements<6>(A, nel); break;
            case 7: dg::run_elements<7>(A, nel); break;
            case 8: dg::run_elements<8>(A, nel); break;
            default: return 4;
        }
    }
    FILE *o = fopen(argv[11], "wb");
    if (!o) return 5;
    fwrite(div.data(), sizeof(double), Np, o);
    if (equal) fwrite(div2.data(), sizeof(double), N, o);
    for (int d = 0; d < 3; ++d) fwrite(g[d].data(), sizeof(double), N, o);
    fclose(o);
    return 0;
}
