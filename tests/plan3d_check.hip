// Host-side check of the 3D work lists (built and run on the CPU by
// tests/test_plan3d_cpu.py; no GPU call is made).  Arguments: nx ny nz P m
// d0x d0y d0z dnx dny dnz g0x g0y g0z gnx gny gnz.  Checks that every
// tile-chunk holding a general plane appears in exactly one list, that no
// other chunk does, that single-axis codes name the one absorber axis the
// chunk's planes need, that the design list holds exactly the chunks that
// meet the design or gap box, and that the plain launch's box holds every
// plain tile-plane.  Prints one summary line; exit status 0 when all hold.
#include "../paper_2203_01462_amd/csrc/fdtd_3d.hip"

#include <cstdio>
#include <cstdlib>

using namespace fdtd;

int main(int argc, char **argv) {
  if (argc != 18) {
    std::fprintf(stderr, "usage: nx ny nz P m d0(3) dn(3) g0(3) gn(3)\n");
    return 2;
  }
  int v[17];
  for (int a = 0; a < 17; ++a) v[a] = std::atoi(argv[a + 1]);
  Step3D<float> p{};
  for (int d = 0; d < 3; ++d) {
    p.n[d] = v[d];
    p.d0[d] = v[5 + d];
    p.dn[d] = v[8 + d];
    p.g0[d] = v[11 + d];
    p.gn[d] = v[14 + d];
  }
  p.P = v[3];
  p.tf_on = 1;
  for (int d = 0; d < 3; ++d) {
    p.lo[d] = v[3] + v[4];
    p.hi[d] = p.n[d] - 1 - v[3] - v[4];
  }
  int nS = 0, nM = 0, nD = 0, axD = 0;
  const std::vector<int> L = gen3d_plan(p, nS, nM, nD, axD);
  const int nbx = (p.n[0] + TX - 1) / TX, nby = (p.n[1] + TY - 1) / TY, nbz = (p.n[2] + KC - 1) / KC;
  const int tot = nbx * nby * nbz;
  int bad = 0;
  if ((int)L.size() != nS + nM + nD || nS % 8 || nM % 8 || nD % 8) ++bad;
  std::vector<int> seen(tot, 0), part(tot, -1), axis(tot, -1);
  for (int i = 0; i < (int)L.size(); ++i) {
    const int pt = i < nS ? 0 : i < nS + nM ? 1 : 2;
    int c = L[i];
    if (c < 0) continue;
    if (pt == 0) {
      axis[c >> 2] = c & 3;
      c >>= 2;
    }
    if (c >= tot) {
      ++bad;
      continue;
    }
    ++seen[c];
    part[c] = pt;
  }
  int general = 0, plain_planes = 0;
  int pb[6];
  plain3d_box(p, pb);
  for (int c = 0; c < tot; ++c) {
    const int bx = c % nbx, by = (c / nbx) % nby, bz = c / (nbx * nby);
    Tile tl = tile_xy(p, bx * TX, by * TY);
    tl.kb = bz * KC;
    tl.ke = std::min(tl.kb + KC, p.n[2]);
    int planes = 0, ax = 0;
    bool have = false;
    for (int k = tl.kb; k < tl.ke; ++k) {
      if (plane_plain(p, tl, k)) {
        have = false;
        ++plain_planes;
        const bool in = bx * TX >= pb[0] && bx * TX < pb[0] + pb[3] && by * TY >= pb[1] && by * TY < pb[1] + pb[4] &&
                        k >= pb[2] && k < pb[2] + pb[5];
        if (!in) ++bad;
        continue;
      }
      if (!have && k >= 1) ax |= plane_axes(p, k - 1);
      ax |= plane_axes(p, k);
      have = true;
      ++planes;
    }
    ax |= tile_axes(p, tl);
    if (planes == 0) {
      if (seen[c]) ++bad;
      continue;
    }
    ++general;
    if (seen[c] != 1) {
      ++bad;
      continue;
    }
    const bool des = design_chunk(p, tl);
    if (des != (part[c] == 2)) ++bad;
    if (part[c] == 0) {
      const int want = ax == 1 ? 0 : ax == 2 ? 1 : ax == 4 ? 2 : ax == 0 ? 3 : -1;
      if (axis[c] != want) ++bad;
    }
    if (part[c] == 1 && (ax == 0 || ax == 1 || ax == 2 || ax == 4)) ++bad;
    if (part[c] == 2 && (ax & ~axD)) ++bad;
  }
  std::printf("chunks %d general %d lists %d %d %d axD %d plain-box %d %d %d %d %d %d plain-planes %d bad %d\n", tot,
              general, nS, nM, nD, axD, pb[0], pb[1], pb[2], pb[3], pb[4], pb[5], plain_planes, bad);
  return bad ? 1 : 0;
}
