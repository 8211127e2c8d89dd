// Host-side check of the 3D work lists (built and run on the CPU by
// tests/test_plan3d_cpu.py; no GPU call is made).  Arguments: nx ny nz P m
// d0x d0y d0z dnx dny dnz g0x g0y g0z gnx gny gnz.  Checks that every
// tile-chunk holding a general plane appears in exactly one list, that no
// other chunk does, that single-axis codes name the one absorber axis the
// chunk's planes need, that the design list holds exactly the chunks that
// meet the design or gap box, that the plain launch's box holds every
// plain tile-plane, and that the two-step super-chunks keep to plain
// background and store every node the per-step launches read from them.
// Prints one summary line; exit status 0 when all hold.
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
  // two-step super-chunks: each flagged chunk once in the launch list; every
  // chunk node in a plain tile-plane and every node within three of the
  // chunk plain background (inside the walls, off the absorber, injection
  // planes, design and gap); every super-chunk node that a node outside the
  // super-chunks reads in a per-step update (its 26 neighbours) stored by the
  // pass's border rule
  for (int a = 0; a < 6; ++a) p.pb[a] = pb[a];
  int so[3], sn[3];
  std::vector<unsigned char> flags;
  const std::vector<int> SL = plan3d_super(p, so, sn, flags);
  const int nx = p.n[0], ny = p.n[1], nz = p.n[2], P = p.P;
  int nsup = 0, sbad = 0;
  std::vector<int> faces_of(flags.size(), -1);
  if (SL.size() % 8) ++sbad;
  for (int code : SL) {
    if (code < 0) continue;
    const int ci = code >> 6;
    if (ci >= (int)flags.size() || !flags[ci] || faces_of[ci] >= 0) {
      ++sbad;
      continue;
    }
    faces_of[ci] = code & 63;
    ++nsup;
  }
  auto plain_node = [&](int i, int j, int k) {
    const int c3[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
      const int v = c3[a], n = p.n[a];
      if (v < 1 || v > n - 2 || pml_e(v, n, P) || pml_h(v, n, P)) return false;
      if (v == p.lo[a] - 1 || v == p.lo[a] || v == p.hi[a] || v == p.hi[a] + 1) return false;
    }
    auto in = [&](const int *o, const int *n) {
      return i >= o[0] && i < o[0] + n[0] && j >= o[1] && j < o[1] + n[1] && k >= o[2] && k < o[2] + n[2];
    };
    return !in(p.d0, p.dn) && !in(p.g0, p.gn);
  };
  std::vector<int> owner((size_t)nx * ny * nz, -1);  // super-chunk of each node
  for (int ci = 0; ci < (int)flags.size(); ++ci) {
    if (!flags[ci]) continue;
    if (faces_of[ci] < 0) ++sbad;  // flagged but not launched
    const int cx = ci % sn[0], cy = (ci / sn[0]) % sn[1], cz = ci / (sn[0] * sn[1]);
    const int a = so[0] + cx * SCX, b = so[1] + cy * SCY, kb = so[2] + cz * SCZ;
    for (int k = kb - 3; k < kb + SCZ + 3; ++k)
      for (int j = b - 3; j < b + SCY + 3; ++j)
        for (int i = a - 3; i < a + SCX + 3; ++i) {
          if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz || !plain_node(i, j, k)) {
            ++sbad;
            continue;
          }
          const bool mine = i >= a && i < a + SCX && j >= b && j < b + SCY && k >= kb && k < kb + SCZ;
          if (!mine) continue;
          const Tile tl = tile_xy(p, i - i % TX, j - j % TY);
          if (!plane_plain(p, tl, k)) ++sbad;
          owner[((size_t)k * ny + j) * nx + i] = ci;
        }
  }
  long long super_nodes = 0;
  for (int k = 1; k < nz - 1; ++k)
    for (int j = 1; j < ny - 1; ++j)
      for (int i = 1; i < nx - 1; ++i) {
        const int ci = owner[((size_t)k * ny + j) * nx + i];
        if (ci < 0) continue;
        ++super_nodes;
        const int f = faces_of[ci];
        if (f < 0) continue;
        const int cx = ci % sn[0], cy = (ci / sn[0]) % sn[1], cz = ci / (sn[0] * sn[1]);
        const int a = so[0] + cx * SCX, b = so[1] + cy * SCY, kb = so[2] + cz * SCZ;
        const bool stored = (i == a && (f & 1)) || (i == a + SCX - 1 && (f & 2)) || (j == b && (f & 4)) ||
                            (j == b + SCY - 1 && (f & 8)) || (k == kb && (f & 16)) || (k == kb + SCZ - 1 && (f & 32));
        bool read_outside = false;
        for (int dk = -1; dk <= 1; ++dk)
          for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di)
              read_outside = read_outside || owner[((size_t)(k + dk) * ny + j + dj) * nx + i + di] < 0;
        if (read_outside && !stored) ++sbad;
      }
  bad += sbad;
  std::printf("chunks %d general %d lists %d %d %d axD %d plain-box %d %d %d %d %d %d plain-planes %d "
              "super %d super-nodes %lld super-bad %d bad %d\n",
              tot, general, nS, nM, nD, axD, pb[0], pb[1], pb[2], pb[3], pb[4], pb[5], plain_planes, nsup, super_nodes,
              sbad, bad);
  return bad ? 1 : 0;
}
