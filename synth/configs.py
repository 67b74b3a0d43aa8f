"""Workload shapes and seeded parameter draws.

Each named configuration fixes the pupil/focal/detector sizes, the aperture,
the Zernike set, the band, the sources, the dithers and the flat-field
statistics. ``make_workload`` draws the truth and the evaluation point from
a fixed seed. The draws follow the paper's experiment (Sections 3-4): the
truth carries random Zernike aberrations and a random pixel response; the
evaluation point is the paper's starting point for its fit -- unaberrated
optics, a uniform pixel response, positions perturbed by N(0, 1 px) and
fluxes scaled by N(1, 0.1).

Photon-noise data needs the model image at the truth, which this package
cannot compute (it holds no optics). ``Workload.with_data`` draws Poisson
counts from an image the caller supplies; ``standin_image`` gives a smooth
image with the right flux and footprint for sizes where computing the truth
in FP64 on the host is too slow.
"""
from __future__ import annotations

import dataclasses
import functools
from dataclasses import dataclass, field

import numpy as np

from .geometry import aperture, binary_phase_screen, keys_bicubic_matrix, zernike_basis

DEFAULT_DIAMETER = 0.5  # metres, the paper's listing in Section 3
CONFIG_NAMES = ("c1", "c2", "c3", "c5")


@dataclass
class Problem:
    """Shape and optics of one forward+gradient problem."""
    n_pupil: int
    n_focal: int
    oversample: int
    wavelengths: np.ndarray          # metres, FP64 [n_wavelengths]
    weights: np.ndarray              # spectral weights, FP64 [n_wavelengths], sum 1
    n_sources: int
    n_frames: int
    n_zernike: int
    n_map: int = 0                   # bicubic nodes per side, 0 = no map
    diameter: float = DEFAULT_DIAMETER
    focal_pixel: float = 0.0         # focal-grid pitch (radians); detector pixel = oversample * this
    obstruction: float = 0.0
    spider_px: float = 0.0
    noll: tuple = ()
    intrapixel: bool = False

    @property
    def n_det(self) -> int:
        return self.n_focal // self.oversample

    @property
    def n_wavelengths(self) -> int:
        return len(self.wavelengths)

    @property
    def n_psf(self) -> int:
        return self.n_frames * self.n_sources * self.n_wavelengths

    @property
    def pupil_pixel(self) -> float:
        return self.diameter / self.n_pupil

    def mft_flops(self) -> float:
        """Real flops of one two-sided MFT (complex MAC = 8 flops), Section 3's two products."""
        ni, no = self.n_pupil, self.n_focal
        return 8.0 * no * ni * (ni + no)


@dataclass
class Workload:
    problem: Problem
    transmission: np.ndarray           # f32 [Ni, Ni]
    zbasis: np.ndarray                 # f32 [Nz, Ni, Ni]
    map_basis: np.ndarray | None       # f32 [Ni, n_map]
    intrapixel: np.ndarray | None      # f32 [Q, Q]
    coeffs_true: np.ndarray            # f32 [Nz]
    map_true: np.ndarray | None        # f32 [n_map, n_map]
    flat_true: np.ndarray              # f32 [Ndet, Ndet]
    sources_true: np.ndarray           # f32 [F, S, 3]: alpha, beta (rad), photons
    coeffs: np.ndarray                 # evaluation point, f32
    phase_map: np.ndarray | None
    flat: np.ndarray
    sources: np.ndarray
    prior_mu: float
    prior_sigma: float
    data: np.ndarray | None = None     # f32 [F, Ndet, Ndet]
    _data_seed: object = field(default=None, repr=False)

    def with_data(self, image: np.ndarray) -> "Workload":
        """Return a copy whose data are Poisson counts of ``image`` [F, Ndet, Ndet]."""
        rng = np.random.default_rng(self._data_seed)
        lam = np.clip(np.asarray(image, dtype=np.float64), 0.0, None)
        d = rng.poisson(lam).astype(np.float32)
        return dataclasses.replace(self, data=d)

    def truth_params(self) -> dict:
        return dict(coeffs=self.coeffs_true, phase_map=self.map_true, flat=self.flat_true,
                    sources=self.sources_true)

    def eval_params(self) -> dict:
        return dict(coeffs=self.coeffs, phase_map=self.phase_map, flat=self.flat, sources=self.sources)


_BASE = {
    # smallest case: unobstructed, monochromatic, Noll 2-11
    "c1": dict(n_pupil=64, n_focal=64, oversample=2, band=(600e-9, 600e-9), n_wavelengths=1,
               noll=tuple(range(2, 12)), zsigma=30e-9, obstruction=0.0, spider_px=0.0,
               sources="single", flux=1e6, n_frames=1, dither=0.0, flat_sigma=0.05, intrapixel=False,
               n_map=0, map_sigma=0.0, centre=600e-9),
    # polychromatic FP32 case
    "c2": dict(n_pupil=256, n_focal=512, oversample=4, band=(500e-9, 700e-9), n_wavelengths=20,
               noll=tuple(range(2, 66)), zsigma=20e-9, obstruction=0.3, spider_px=2.0,
               sources="single", flux=1e8, n_frames=1, dither=0.0, flat_sigma=0.03, intrapixel=False,
               n_map=0, map_sigma=0.0, centre=600e-9),
    # dithered binary, intra-pixel gradient
    "c3": dict(n_pupil=512, n_focal=768, oversample=3, band=(500e-9, 700e-9), n_wavelengths=32,
               noll=tuple(range(2, 130)), zsigma=20e-9, obstruction=0.3, spider_px=2.0,
               sources="binary", flux=1e8, n_frames=64, dither=4.0, flat_sigma=0.05, intrapixel=True,
               n_map=0, map_sigma=0.0, centre=600e-9),
    # millions of flat-field parameters, Zernikes + bicubic map
    "c5": dict(n_pupil=1024, n_focal=2048, oversample=2, band=(500e-9, 700e-9), n_wavelengths=16,
               noll=tuple(range(2, 258)), zsigma=5e-9, obstruction=0.3, spider_px=2.0,
               sources="single", flux=1e8, n_frames=16, dither=4.0, flat_sigma=0.05, intrapixel=False,
               n_map=64, map_sigma=5e-9, centre=600e-9),
}
_SEED_INDEX = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4}


def _spec(name: str, overrides: dict) -> dict:
    base = name.split("-")[0]
    spec = dict(_BASE[base])
    for k, v in overrides.items():
        if k not in spec:
            raise KeyError(f"unknown override {k!r}")
        spec[k] = v
    return spec


def make_problem(name: str, **overrides) -> Problem:
    """Problem of configuration ``name`` ("c1", "c2", "c3", "c5"), sizes optionally overridden."""
    s = _spec(name, overrides)
    lo, hi = s["band"]
    nl = s["n_wavelengths"]
    lam = np.linspace(lo, hi, nl) if nl > 1 else np.array([0.5 * (lo + hi)])
    Q = s["oversample"]
    if s["n_focal"] % Q:
        raise ValueError("n_focal must be a multiple of the oversampling factor")
    det_pix = s["centre"] / (2.0 * DEFAULT_DIAMETER)   # Nyquist at band centre
    n_src = 1 if s["sources"] == "single" else 2
    return Problem(n_pupil=s["n_pupil"], n_focal=s["n_focal"], oversample=Q, wavelengths=lam,
                   weights=np.full(nl, 1.0 / nl), n_sources=n_src, n_frames=s["n_frames"],
                   n_zernike=len(s["noll"]), n_map=s["n_map"], diameter=DEFAULT_DIAMETER,
                   focal_pixel=det_pix / Q, obstruction=s["obstruction"], spider_px=s["spider_px"],
                   noll=tuple(s["noll"]), intrapixel=s["intrapixel"])


def intrapixel_kernel(Q: int) -> np.ndarray:
    """Fixed intra-pixel response: 0.5% peak-to-peak gradient along x, mean 1."""
    b = np.arange(Q, dtype=np.float64)
    row = 1.0 + 0.005 * (b - (Q - 1) / 2.0) / max(Q - 1, 1)
    return np.tile(row, (Q, 1))


def make_workload(name: str, **overrides) -> Workload:
    """Seeded truth, evaluation point and static inputs of configuration ``name``.

    Seeds come from ``SeedSequence([2406, 8703, k])`` with ``k`` the config's
    index; its children are used in a fixed order: Zernike truth, flat truth,
    sources, dithers, Poisson data, evaluation-point perturbation, bicubic map.
    """
    s = _spec(name, overrides)
    P = make_problem(name, **overrides)
    ss = np.random.SeedSequence([2406, 8703, _SEED_INDEX[name.split("-")[0]]])
    ch = ss.spawn(8)
    rz, rf, rs, rd, rpois, rinit, rmap = (np.random.default_rng(c) for c in ch[:7])
    Ni, Nd, Q = P.n_pupil, P.n_det, P.oversample
    D = P.diameter
    trans = aperture(Ni, D, P.obstruction, P.spider_px)
    zb = zernike_basis(list(P.noll), Ni, D)
    coeffs_true = rz.normal(0.0, s["zsigma"], P.n_zernike)
    flat_true = 1.0 + s["flat_sigma"] * rf.normal(size=(Nd, Nd))
    det_pix = P.focal_pixel * Q
    lam_c = s["centre"]
    if s["sources"] == "single":
        pos = np.zeros((1, 2))
        flux = np.array([s["flux"]])
    else:  # binary: separation 10 lambda_c/D, flux ratio 0.3, random position angle
        sep = 10.0 * lam_c / D
        pa = rs.uniform(0.0, 2.0 * np.pi)
        half = 0.5 * sep * np.array([np.cos(pa), np.sin(pa)])
        pos = np.stack([-half, half])
        f1 = s["flux"] / 1.3
        flux = np.array([f1, 0.3 * f1])
    F = P.n_frames
    dith = rd.uniform(-s["dither"], s["dither"], size=(F, 2)) * det_pix if s["dither"] > 0 else np.zeros((F, 2))
    src_true = np.zeros((F, P.n_sources, 3))
    src_true[:, :, 0:2] = pos[None, :, :] + dith[:, None, :]
    src_true[:, :, 2] = flux[None, :]
    # evaluation point: positions + N(0, 1 px), fluxes x N(1, 0.1), no aberration, uniform flat
    dpos = rinit.normal(0.0, 1.0, size=(P.n_sources, 2)) * det_pix
    fscale = rinit.normal(1.0, 0.1, size=P.n_sources)
    src_eval = src_true.copy()
    src_eval[:, :, 0:2] += dpos[None, :, :]
    src_eval[:, :, 2] *= fscale[None, :]
    if P.n_map:
        mb = keys_bicubic_matrix(Ni, P.n_map, D)
        map_true = rmap.normal(0.0, s["map_sigma"], size=(P.n_map, P.n_map))
        map_eval = np.zeros_like(map_true)
    else:
        mb = map_true = map_eval = None
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return Workload(problem=P, transmission=f32(trans), zbasis=f32(zb), map_basis=f32(mb),
                    intrapixel=f32(intrapixel_kernel(Q)) if P.intrapixel else None,
                    coeffs_true=f32(coeffs_true), map_true=f32(map_true), flat_true=f32(flat_true),
                    sources_true=f32(src_true), coeffs=np.zeros(P.n_zernike, np.float32),
                    phase_map=f32(map_eval), flat=np.ones((Nd, Nd), np.float32), sources=f32(src_eval),
                    prior_mu=1.0, prior_sigma=float(s["flat_sigma"]), _data_seed=ch[4])


def standin_image(w: Workload) -> np.ndarray:
    """Smooth data-like image [F, Ndet, Ndet]: one Gaussian blob per source.

    Each blob has the source's flux, width 0.45 lambda_c/D and sits at the
    source's true position, times the true flat field. It is a stand-in for
    the truth model where computing that in FP64 on the host is too slow;
    it is not a model of the optics.
    """
    P = w.problem
    det_pix = P.focal_pixel * P.oversample
    xd = (np.arange(P.n_det) - (P.n_det - 1) / 2.0) * det_pix
    sig = 0.45 * float(np.mean(P.wavelengths)) / P.diameter
    out = np.zeros((P.n_frames, P.n_det, P.n_det))
    for f in range(P.n_frames):
        for s in range(P.n_sources):
            a, b, phi = (float(v) for v in w.sources_true[f, s])
            gx = np.exp(-0.5 * ((xd - a) / sig) ** 2)
            gy = np.exp(-0.5 * ((xd - b) / sig) ** 2)
            img = np.outer(gy, gx)
            out[f] += phi * img / img.sum()
    return out * w.flat_true[None].astype(np.float64) + 1.0


def make_c4_workloads(n_problems: int = 128, scale: float = 1.0) -> list:
    """Independent uneven fits of the batched configuration, drawn from seed child 7.

    Per problem: pupil N_i from {128, 192, 256, 384, 512}, focal N_o from
    {64, 128, 256} at oversampling Q ~ U{2, 3, 4} with N_det = floor(N_o / Q)
    and N_o := Q N_det (so 63, 126 and 255 occur), 8-64 wavelengths in
    450-800 nm, 16-128 Zernikes ~N(0, 25 nm), 1-3 stars with positions
    U(-N_det/4, N_det/4) px and fluxes log-uniform in [1e6, 1e8], one frame,
    the 30%-obstructed aperture with spiders, flat ~N(1, 0.05), detector pixel
    Nyquist at 625 nm. ``scale`` < 1 shrinks the sizes (pupil, focal grid,
    wavelengths, Zernikes) for tests that compare every problem with the oracle.
    """
    ss = np.random.SeedSequence([2406, 8703, _SEED_INDEX["c4"]])
    size_rng = np.random.default_rng(ss.spawn(8)[7])
    out = []
    for k in range(n_problems):
        ni = int(size_rng.choice([128, 192, 256, 384, 512]))
        no = int(size_rng.choice([64, 128, 256]))
        q = int(size_rng.integers(2, 5))
        nl = int(size_rng.integers(8, 65))
        nz = int(size_rng.integers(16, 129))
        ns = int(size_rng.integers(1, 4))
        if scale != 1.0:
            ni = max(16, int(round(ni * scale / 8)) * 8)
            no = max(2 * q, int(no * scale))
            nl = max(1, int(round(nl * scale)))
            nz = max(2, int(round(nz * scale)))
        nd = no // q
        no = q * nd
        out.append(_c4_problem(k, ni, no, q, nl, nz, ns))
    return out


@functools.lru_cache(maxsize=None)
def _c4_static(ni: int):
    """Aperture and the Noll 2..129 basis of one pupil size (shared by every problem of that size)."""
    D = DEFAULT_DIAMETER
    return (np.ascontiguousarray(aperture(ni, D, 0.3, 2.0), dtype=np.float32),
            np.ascontiguousarray(zernike_basis(list(range(2, 130)), ni, D), dtype=np.float32))


def _c4_problem(k, ni, no, q, nl, nz, ns) -> Workload:
    ss = np.random.SeedSequence([2406, 8703, _SEED_INDEX["c4"], k])
    rz, rf, rs, rpois, rinit = (np.random.default_rng(c) for c in ss.spawn(5))
    D, lam_c = DEFAULT_DIAMETER, 625e-9
    det_pix = lam_c / (2.0 * D)
    lam = np.linspace(450e-9, 800e-9, nl) if nl > 1 else np.array([lam_c])
    noll = tuple(range(2, nz + 2))
    P = Problem(n_pupil=ni, n_focal=no, oversample=q, wavelengths=lam, weights=np.full(nl, 1.0 / nl), n_sources=ns,
                n_frames=1, n_zernike=nz, diameter=D, focal_pixel=det_pix / q, obstruction=0.3, spider_px=2.0,
                noll=noll)
    nd = P.n_det
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    pos = rs.uniform(-nd / 4, nd / 4, size=(ns, 2)) * det_pix
    flux = 10 ** rs.uniform(6, 8, size=ns)
    src_true = np.zeros((1, ns, 3))
    src_true[0, :, :2] = pos
    src_true[0, :, 2] = flux
    src_eval = src_true.copy()
    src_eval[0, :, :2] += rinit.normal(0.0, 1.0, size=(ns, 2)) * det_pix
    src_eval[0, :, 2] *= rinit.normal(1.0, 0.1, size=ns)
    trans, basis = _c4_static(ni)
    return Workload(problem=P, transmission=trans, zbasis=np.ascontiguousarray(basis[:nz]),
                    map_basis=None, intrapixel=None, coeffs_true=f32(rz.normal(0.0, 25e-9, nz)), map_true=None,
                    flat_true=f32(1.0 + 0.05 * rf.normal(size=(nd, nd))), sources_true=f32(src_true),
                    coeffs=np.zeros(nz, np.float32), phase_map=None, flat=np.ones((nd, nd), np.float32),
                    sources=f32(src_eval), prior_mu=1.0, prior_sigma=0.05, _data_seed=ss.spawn(6)[5])


@dataclass
class DitheredWorkload:
    """One scene imaged in several frames offset by whole detector pixels (the paper's run, Section 3).

    The PSFs are those of an enlarged plane: ``problem`` has n_focal =
    Q (n_det + 2 margin) and one frame; frame f is the window of that plane
    shifted by ``dithers[f]`` = (dx, dy) detector pixels. Sources are shared
    by all frames: [S, 3] = alpha, beta (radians), photons per frame.
    """
    problem: Problem
    n_det: int
    margin: int
    dithers: np.ndarray                # int32 [F, 2]
    transmission: np.ndarray
    zbasis: np.ndarray
    coeffs_true: np.ndarray
    flat_true: np.ndarray              # [n_det, n_det]
    sources_true: np.ndarray           # [S, 3]
    coeffs: np.ndarray
    flat: np.ndarray
    sources: np.ndarray
    prior_mu: float
    prior_sigma: float
    map_basis: np.ndarray | None = None
    intrapixel: np.ndarray | None = None
    phase_screen: np.ndarray | None = None  # [n_pupil, n_pupil] static phase, radians
    data: np.ndarray | None = None     # [F, n_det, n_det]
    _data_seed: object = field(default=None, repr=False)

    @property
    def n_frames(self) -> int:
        return len(self.dithers)

    def per_frame_sources(self, sources) -> np.ndarray:
        """[F, S, 3] sources of the equivalent per-frame problem: dither added to every position."""
        src = np.repeat(np.asarray(sources, np.float64)[None], self.n_frames, axis=0)
        pix = self.problem.focal_pixel * self.problem.oversample
        src[:, :, 0] += self.dithers[:, 0][:, None] * pix
        src[:, :, 1] += self.dithers[:, 1][:, None] * pix
        return src.astype(np.float32)

    def with_data(self, image: np.ndarray) -> "DitheredWorkload":
        rng = np.random.default_rng(self._data_seed)
        lam = np.clip(np.asarray(image, dtype=np.float64), 0.0, None)
        return dataclasses.replace(self, data=rng.poisson(lam).astype(np.float32))

    def eval_params(self) -> dict:
        return dict(coeffs=self.coeffs, phase_map=None, flat=self.flat, sources=self.sources)

    def truth_params(self) -> dict:
        return dict(coeffs=self.coeffs_true, phase_map=None, flat=self.flat_true, sources=self.sources_true)


_P0 = dict(n_pupil=512, n_det=1024, oversample=1, margin=20, wavelengths=(545e-9, 595e-9, 645e-9), n_sources=20,
           noll=tuple(range(4, 11)), zsigma=20e-9, inner_radius=0.1, det_pixel_mas=12.0, flat_sigma=0.1,
           flux=(1e7, 1e8),
           dithers=((0, 0), (20, 20), (20, -20), (-20, 20), (-20, -20)), mask=True)


def make_dithered_workload(**overrides) -> DitheredWorkload:
    """The paper's own run (Section 3) as synthetic inputs: 20 stars, 3 wavelengths, 7 Zernikes
    (Noll 4-10, 20 nm), a 512-pixel pupil with a central obstruction of radius D/10, a 1024-pixel
    detector of 12 mas pixels, a pixel response 1 + 0.1 N(0, 1), and 5 frames: undithered and
    dithered by (+-20, +-20) pixels, all from one 1064-pixel plane. Stars are placed uniformly
    at least ``margin`` + 12 pixels inside the detector, fluxes log-uniform in ``flux``. Sizes can be
    overridden for tests. The paper's binary phase plate (its mask file is not available) is
    stood in for by ``binary_phase_screen`` (``mask=False`` leaves it out). Seeds:
    ``SeedSequence([2406, 8703, 5])``, children in the order Zernike truth, flat truth, sources,
    (unused), Poisson data, evaluation-point perturbation, phase plate.
    """
    s = dict(_P0)
    for k, v in overrides.items():
        if k not in s:
            raise KeyError(f"unknown override {k!r}")
        s[k] = v
    ss = np.random.SeedSequence([2406, 8703, 5])
    ch = ss.spawn(8)
    rz, rf, rs, _, rpois, rinit, rmask = (np.random.default_rng(c) for c in ch[:7])
    Ni, Nd, Q, m = s["n_pupil"], s["n_det"], s["oversample"], s["margin"]
    lam = np.asarray(s["wavelengths"], np.float64)
    det_pix = s["det_pixel_mas"] * np.pi / 180 / 3600 / 1000
    D = DEFAULT_DIAMETER
    S = s["n_sources"]
    P = Problem(n_pupil=Ni, n_focal=Q * (Nd + 2 * m), oversample=Q, wavelengths=lam,
                weights=np.full(len(lam), 1.0 / len(lam)), n_sources=S, n_frames=1, n_zernike=len(s["noll"]),
                diameter=D, focal_pixel=det_pix / Q, obstruction=2 * s["inner_radius"], spider_px=0.0,
                noll=tuple(s["noll"]))
    trans = aperture(Ni, D, P.obstruction, 0.0)
    zb = zernike_basis(list(P.noll), Ni, D)
    coeffs_true = rz.normal(0.0, s["zsigma"], P.n_zernike)
    flat_true = 1.0 + s["flat_sigma"] * rf.normal(size=(Nd, Nd))
    lim = max(Nd / 2 - m - 12, 1.0)
    pos = rs.uniform(-lim, lim, size=(S, 2)) * det_pix
    lo, hi = np.log10(s["flux"][0]), np.log10(s["flux"][1])
    flux = 10 ** rs.uniform(lo, hi, size=S)
    src_true = np.concatenate([pos, flux[:, None]], axis=1)
    src_eval = src_true.copy()
    src_eval[:, :2] += rinit.normal(0.0, 1.0, size=(S, 2)) * det_pix
    src_eval[:, 2] *= rinit.normal(1.0, 0.1, size=S)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return DitheredWorkload(problem=P, n_det=Nd, margin=m, dithers=np.asarray(s["dithers"], np.int32),
                            transmission=f32(trans), zbasis=f32(zb), coeffs_true=f32(coeffs_true),
                            flat_true=f32(flat_true), sources_true=f32(src_true),
                            coeffs=np.zeros(P.n_zernike, np.float32), flat=np.ones((Nd, Nd), np.float32),
                            sources=f32(src_eval), prior_mu=1.0, prior_sigma=float(s["flat_sigma"]),
                            phase_screen=binary_phase_screen(Ni, rmask) if s["mask"] else None,
                            _data_seed=ch[4])


def dithered_standin_image(w: DitheredWorkload) -> np.ndarray:
    """Smooth stand-in image [F, n_det, n_det] (one Gaussian per star at its dithered true position)."""
    P = w.problem
    det_pix = P.focal_pixel * P.oversample
    xd = (np.arange(w.n_det) - (w.n_det - 1) / 2.0) * det_pix
    sig = 0.45 * float(np.mean(P.wavelengths)) / P.diameter
    src = w.per_frame_sources(w.sources_true)
    out = np.zeros((w.n_frames, w.n_det, w.n_det))
    for f in range(w.n_frames):
        for a, b, phi in src[f].astype(np.float64):
            img = np.outer(np.exp(-0.5 * ((xd - b) / sig) ** 2), np.exp(-0.5 * ((xd - a) / sig) ** 2))
            out[f] += phi * img / max(img.sum(), 1e-300)
    return out * w.flat_true[None].astype(np.float64) + 1.0
