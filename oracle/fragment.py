"""Fragmentation of the collapsed medium into halos (oracle; test infrastructure only).

Section "Fragmentation": grid points ("particles") are taken in decreasing F_max, which is
chronological order; each one looks at its six neighbours and the halos they belong to:

  (i)   no neighbour has collapsed yet: the particle is a peak and starts a new halo;
  (ii)  the neighbours touch one halo: particle and halo are displaced with the Zel'dovich
        approximation and the particle is accreted if their distance is below the accretion
        threshold (eq. accretion), else it becomes a filament particle; after an accretion every
        neighbour tagged as filament joins the halo too;
  (iii) the neighbours touch several halos: accretion is tried on the halo with the smallest d/R,
        then every pair of touched halos is merged if their displaced distance is below the
        merging threshold (eq. merging), and if the particle was not accreted, accretion is tried
        again after the mergers;
  (iv)  the neighbours touch filament particles only: the particle becomes a filament particle.

Readings (the paper leaves these open or garbled):
* particles with F_max >= f_min take part (f_min = 1/D at the output time); ties in F_max are
  taken in increasing linear index;
* the time of an event is the growing mode of the particle being processed, D = 1/F_max;
* Zel'dovich displacement: x = q + D u with u = v_max (the smoothed displacement recorded at R_max)
  in grid units, positions in grid units, periodic with the minimum image;
* a halo keeps the number of particles N_h, the sum of its members' minimum-image offsets from the
  particle that founded it, and the sum of their u; its displaced position is
  q_founder + (sum of offsets) / N_h + D (sum of u) / N_h;
* halo radius R = (3 N_h / 4 pi)^(1/3) in grid units (the printed sqrt(N_h) x 3/4pi is garbled);
* sigma(R) is the linear rms of the field smoothed with a top-hat of radius R (R L / N Mpc/h),
  from the field's spectrum, times D ("computed at the collapse time"); it is tabulated at 64
  radii per octave from the radius of one particle up and interpolated linearly in ln R;
* the merging constant is Table 1's f_rm (printed as f_ma in eq. merging);
* accretion uses the threshold f_a R + f_ra + f_s (R sigma)^1.7 with R of the halo before the
  particle joins; merging d < f_m max(R1, R2) + f_rm;
* case (iii): touched halos are taken in increasing halo id; pairs (a, b), a < b, in that order,
  each with the halos as updated by earlier mergers; the merged halo keeps the id of the larger
  (the smaller id on equal sizes); the retried accretion uses the smallest d/R over the distinct
  merged halos;
* the smallest d/R picks the first halo in id order on equal values;
* a halo's id is the linear index of the particle that founded it.

Output per particle: NOT_COLLAPSED (-2), FILAMENT (-1), or the id of its halo; and N_h per halo.
The catalogue (the halo output the section describes: masses, Lagrangian centres of mass, Zel'dovich
displacements) lists, per halo in increasing id, N_h, the centre of mass q_founder + offsets/N_h
wrapped into [0, N) and times the cell size (Mpc/h), and the mean displacement u_sum/N_h times the
cell size (Mpc/h at D = 1).  The merger history (reported at the final time: the masses of the
merging halos at each merger) lists every merger in the order it happened: the F_max of the particle
whose step caused it, the id and N_h of the halo that keeps its id, and those of the one absorbed.
"""

import numpy as np

from . import spectrum

NOT_COLLAPSED = -2
FILAMENT = -1

TABLE1 = {"f_a": 0.285, "f_ra": 0.180, "f_s": 0.060, "f_m": 0.350, "f_rm": 0.700}

NODES_PER_OCTAVE = 64


def halo_radius(nh):
    return (3.0 * nh / (4.0 * np.pi)) ** (1.0 / 3.0)


class SigmaTable:
    """sigma(R) of the linear field (top-hat, z = 0) at R in grid units: nodes R_k = R(1) 2^(k/64),
    linear interpolation in ln R."""

    def __init__(self, n, box, sigma8, gamma, ns, nh_max):
        amp = spectrum.amplitude_for_sigma8(sigma8, gamma, ns)
        self.r0 = halo_radius(1)
        self.step = np.log(2.0) / NODES_PER_OCTAVE
        count = int(np.ceil(np.log(halo_radius(nh_max) / self.r0) / self.step)) + 2
        cell = box / n
        radii = self.r0 * np.exp(np.arange(count) * self.step) * cell
        self.values = np.sqrt(spectrum.sigma2_tophat_many(radii, gamma, ns, amp))

    def __call__(self, r):
        t = np.log(r / self.r0) / self.step
        k = min(int(np.floor(t)), len(self.values) - 2)
        w = t - k
        return self.values[k] + w * (self.values[k + 1] - self.values[k])


def _wrap(d, n):
    """Minimum image of a coordinate difference on a periodic axis of n cells."""
    return d - n * np.floor(d / n + 0.5)


def fragment(F, u, f_min, n, sigma, params=TABLE1, catalog_cell=None, want_mergers=False):
    """Sequential fragmentation.

    F: (N^3,) inverse collapse times; u: (3, N^3) displacements in grid units at D = 1;
    sigma: callable R -> sigma(R) at D = 1.  Returns (label (N^3,) int64, nh dict id -> N_h), and
    with catalog_cell (the cell size in Mpc/h) also the catalogue: (ids, N_h, centre (3, H),
    displacement (3, H)) in increasing id, and with want_mergers the merger list
    [(F, keep, gone, N_keep before, N_gone)] in the order the mergers happened (appended last).
    """
    F = np.asarray(F, dtype=np.float64).ravel()
    u = np.asarray(u, dtype=np.float64).reshape(3, -1)
    fa, fra, fs, fm, frm = (params[k] for k in ("f_a", "f_ra", "f_s", "f_m", "f_rm"))
    vol = n ** 3
    label = np.full(vol, NOT_COLLAPSED, dtype=np.int64)
    parent = {}
    nh, sq, su = {}, {}, {}
    mergers = []

    idx = np.nonzero(F >= f_min)[0]
    order = idx[np.lexsort((idx, -F[idx]))]       # F descending, then index ascending

    def coords(i):
        return np.array([i // (n * n), (i // n) % n, i % n], dtype=np.float64)

    def find(h):
        while parent[h] != h:
            h = parent[h]
        return h

    def position(h, D):
        c = coords(h) + sq[h] / nh[h]
        return c + D * (su[h] / nh[h])

    def dist(a, b):
        d = _wrap(a - b, n)
        return np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])

    def accretion_ok(d, h, D):
        r = halo_radius(nh[h])
        return d < fa * r + fra + fs * (r * sigma(r) * D) ** 1.7

    def add(h, j):
        nh[h] += 1
        sq[h] = sq[h] + _wrap(coords(j) - coords(h), n)
        su[h] = su[h] + u[:, j]
        label[j] = h

    def accrete(i, h, nbrs):
        add(h, i)
        for j in nbrs:
            if label[j] == FILAMENT:
                add(h, j)

    def best_halo(halos, xi, D):
        best, best_v, best_d = None, None, None
        for h in halos:
            d = dist(xi, position(h, D))
            v = d / halo_radius(nh[h])
            if best is None or v < best_v:
                best, best_v, best_d = h, v, d
        return best, best_d

    for i in order:
        D = 1.0 / F[i]
        q = coords(i)
        x, y, z = int(q[0]), int(q[1]), int(q[2])
        nbrs = [((x + 1) % n) * n * n + y * n + z, ((x - 1) % n) * n * n + y * n + z,
                x * n * n + ((y + 1) % n) * n + z, x * n * n + ((y - 1) % n) * n + z,
                x * n * n + y * n + (z + 1) % n, x * n * n + y * n + (z - 1) % n]
        halos = sorted({find(int(label[j])) for j in nbrs if label[j] >= 0})
        has_fil = any(label[j] == FILAMENT for j in nbrs)
        xi = q + D * u[:, i]
        if not halos and not has_fil:                                   # (i)
            parent[i] = i
            nh[i] = 1
            sq[i] = np.zeros(3)
            su[i] = u[:, i].copy()
            label[i] = i
        elif not halos:                                                 # (iv)
            label[i] = FILAMENT
        elif len(halos) == 1:                                           # (ii)
            h = halos[0]
            if accretion_ok(dist(xi, position(h, D)), h, D):
                accrete(i, h, nbrs)
            else:
                label[i] = FILAMENT
        else:                                                           # (iii)
            h, d = best_halo(halos, xi, D)
            accreted = accretion_ok(d, h, D)
            if accreted:
                accrete(i, h, nbrs)
            for a in range(len(halos)):
                for b in range(a + 1, len(halos)):
                    ha, hb = find(halos[a]), find(halos[b])
                    if ha == hb:
                        continue
                    dab = dist(position(ha, D), position(hb, D))
                    if dab < fm * max(halo_radius(nh[ha]), halo_radius(nh[hb])) + frm:
                        keep, gone = (ha, hb) if (nh[ha], -ha) >= (nh[hb], -hb) else (hb, ha)
                        mergers.append((F[i], keep, gone, nh[keep], nh[gone]))
                        off = _wrap(coords(gone) - coords(keep), n)
                        sq[keep] = sq[keep] + sq[gone] + nh[gone] * off
                        su[keep] = su[keep] + su[gone]
                        nh[keep] += nh[gone]
                        parent[gone] = keep
            if not accreted:
                roots = sorted({find(h0) for h0 in halos})
                h, d = best_halo(roots, xi, D)
                if accretion_ok(d, h, D):
                    accrete(i, h, nbrs)
                else:
                    label[i] = FILAMENT

    for j in np.nonzero(label >= 0)[0]:
        label[j] = find(int(label[j]))
    sizes = {h: nh[h] for h in parent if parent[h] == h}
    extra = ()
    if want_mergers:
        extra = (mergers,)
    if catalog_cell is None:
        return (label, sizes) + extra
    ids = np.array(sorted(sizes), dtype=np.int64)
    cnt = np.array([nh[h] for h in ids], dtype=np.int64)
    centre = np.zeros((3, len(ids)))
    disp = np.zeros((3, len(ids)))
    for k, h in enumerate(ids):
        c = coords(h) + sq[h] / nh[h]
        centre[:, k] = (c - n * np.floor(c / n)) * catalog_cell
        disp[:, k] = su[h] / nh[h] * catalog_cell
    return (label, sizes, (ids, cnt, centre, disp)) + extra
