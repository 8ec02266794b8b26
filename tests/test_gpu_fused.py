"""The tile-local form of scoring (sum tables built per tile in LDS from the
frame, sncc_score_frame) against the oracle: rho within 1e-5 at every
offset, the exact window energy n * sum f^2 - (sum f)^2 bit for bit, the
degenerate flags, on ragged tile edges, odd widths (byte loads), the widest
and the tallest templates the form takes, a 128 x 128 template, and the
single-frame workloads at full size; the global form of the same call for
comparison, and the form chosen or refused by size."""

import numpy as np
import pytest

import oracle as O
from workloads import synth

from gpu_util import lib_templates
from oracle_pool import OraclePool

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def S():
    import paper_2502_01286_amd as S
    return S


@pytest.fixture(scope="module")
def ctx(S):
    import torch
    torch.cuda.init()
    c = S.sncc_ctx_create(0)
    yield c
    S.sncc_ctx_destroy(c)


@pytest.fixture(scope="module")
def pool():
    p = OraclePool()
    yield p
    p.close()


def _run(S, ctx, f, t, sigma, form, k_max=5000):
    import torch
    N, M = f.shape
    H, W = t.shape
    tm = lib_templates(S, ctx, [t], [sigma], k_max)
    nu, nv = M - W + 1, N - H + 1
    pitch = nu + 3                                  # a row pitch above the minimum
    rho = torch.full((nv, pitch), 9.0, dtype=torch.float32, device="cuda")
    deg = torch.full((nv, pitch), 7, dtype=torch.uint8, device="cuda")
    en = torch.full((nv, pitch), -1, dtype=torch.int64, device="cuda")
    d = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    used = S.sncc_score_frame(ctx, tm, 0, d, rho, form=form, degen=deg, energy=en)
    S.sncc_sync(ctx)
    S.sncc_tmpl_destroy(tm)
    r, g, e = rho.cpu().numpy(), deg.cpu().numpy(), en.cpu().numpy()
    assert (r[:, nu:] == 9.0).all() and (g[:, nu:] == 7).all() and (e[:, nu:] == -1).all()
    return used, r[:, :nu].astype(np.float64), g[:, :nu], e[:, :nu]


def _check(S, f, t, sigma, used, rho, deg, en, want=None, k_max=5000):
    ta = O.precompute_template_approximation(t, sigma, k_max)
    s, s2 = O.sum_tables(f)
    nv, nu = rho.shape
    vv, uu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    _, _, V = O.window_sums(s, s2, ta.W, ta.H, uu, vv)
    if want is None:
        want = O.rho_map(f, ta, tables=(s, s2))
    assert np.array_equal(en, V)                    # exact energy, bit for bit
    assert np.array_equal(deg, (V == 0).astype(np.uint8))
    err = float(np.abs(rho - want).max())
    assert err <= TOL32, err
    return err


CASES = [
    # (label, frame M x N, template W x H, sigma)
    ("ragged", 203, 77, 13, 9, 6),             # 191 x 69 offsets: partial tiles both ways
    ("odd_width", 151, 60, 20, 16, 8),         # M odd: rows of bytes, not words
    ("tiny_template", 70, 40, 2, 3, 1),
    ("wide", 700, 40, 447, 6, 20),             # widest pitch class
    ("tall", 90, 400, 12, 300, 20),            # rows of LDS near the limit
    ("t128", 400, 300, 128, 128, 4),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tile_local_parity(S, ctx, case):
    label, M, N, W, H, sigma = case
    print("case", label, flush=True)
    f = synth.scene(8100 + M, M, N) if label != "t128" else synth.texture(8100, M, N)
    rng = np.random.default_rng(M + N)
    t, _, _ = synth.crop_template(rng, f, W, H, sigma_max=sigma)
    used, rho, deg, en = _run(S, ctx, f, t, sigma, S.SNCC_FORM_TILE_LOCAL)
    assert used == S.SNCC_FORM_TILE_LOCAL
    e_loc = _check(S, f, t, sigma, used, rho, deg, en)
    used_g, rho_g, deg_g, en_g = _run(S, ctx, f, t, sigma, S.SNCC_FORM_GLOBAL)
    assert used_g == S.SNCC_FORM_GLOBAL
    e_glob = _check(S, f, t, sigma, used_g, rho_g, deg_g, en_g)
    assert np.array_equal(en, en_g) and np.array_equal(deg, deg_g)
    print(f"  max|drho| tile-local {e_loc:.2e}, global {e_glob:.2e}", flush=True)


def test_uniform_region_is_degenerate(S, ctx):
    f = synth.scene(8200, 160, 90)
    f[20:70, 30:120] = 77                          # windows inside are uniform
    rng = np.random.default_rng(5)
    t, _, _ = synth.crop_template(rng, f, 16, 12, sigma_max=6)
    used, rho, deg, en = _run(S, ctx, f, t, 6, S.SNCC_FORM_TILE_LOCAL)
    assert used == S.SNCC_FORM_TILE_LOCAL
    _check(S, f, t, 6, used, rho, deg, en)
    assert deg[30, 50] == 1 and rho[30, 50] == 0.0 and en[30, 50] == 0


def test_form_choice_by_size(S, ctx):
    import torch
    f = synth.scene(8300, 700, 500)
    rng = np.random.default_rng(6)
    t, _, _ = synth.crop_template(rng, f, 300, 250, sigma_max=16)  # n above one exact box
    tm = lib_templates(S, ctx, [t], [16])
    rho = torch.zeros((251, 401), dtype=torch.float32, device="cuda")
    d = torch.from_numpy(f).cuda()
    with pytest.raises(S.SnccError) as e:
        S.sncc_score_frame(ctx, tm, 0, d, rho, form=S.SNCC_FORM_TILE_LOCAL)
    assert e.value.code == S.SNCC_ERANGE
    assert S.sncc_score_frame(ctx, tm, 0, d, rho) == S.SNCC_FORM_GLOBAL
    # automatic choice: tile-local for few segments on a small frame
    # (461 x 653 offsets), global for many
    for sg, want_form in ((40, S.SNCC_FORM_TILE_LOCAL), (2, S.SNCC_FORM_GLOBAL)):
        t2, _, _ = synth.crop_template(rng, f, 48, 40, sigma_max=sg)
        tm2 = lib_templates(S, ctx, [t2], [sg])
        K = S.sncc_tmpl_info(tm2, 0)[2]
        assert (K <= 40) == (want_form == S.SNCC_FORM_TILE_LOCAL), K
        r2 = torch.zeros((500 - 40 + 1, 700 - 48 + 1), dtype=torch.float32, device="cuda")
        assert S.sncc_score_frame(ctx, tm2, 0, d, r2) == want_form
        S.sncc_sync(ctx)
        S.sncc_tmpl_destroy(tm2)
    # a frame of more than 2^19 offsets takes the global form at any K
    fb = synth.scene(8301, 1920, 1080)
    t3, _, _ = synth.crop_template(np.random.default_rng(61), fb, 64, 64, sigma_max=16)
    tm3 = lib_templates(S, ctx, [t3], [16])
    assert S.sncc_tmpl_info(tm3, 0)[2] <= 40
    r3 = torch.zeros((1080 - 64 + 1, 1920 - 64 + 1), dtype=torch.float32, device="cuda")
    db = torch.from_numpy(fb).cuda()
    assert S.sncc_score_frame(ctx, tm3, 0, db, r3) == S.SNCC_FORM_GLOBAL
    S.sncc_sync(ctx)
    S.sncc_tmpl_destroy(tm3)
    S.sncc_sync(ctx)
    S.sncc_tmpl_destroy(tm)
    ta = O.precompute_template_approximation(t, 16)
    rng2 = np.random.default_rng(7)
    us, vs = rng2.integers(0, 401, 300), rng2.integers(0, 251, 300)
    want = O.rho_at(*O.sum_tables(f), ta, us, vs)
    assert np.abs(rho.cpu().numpy()[vs, us] - want).max() <= TOL32


@pytest.mark.parametrize("sigma", [16, 8, 4])
def test_scene_1920x1080_tile_local(S, ctx, pool, sigma):
    wl = synth.scene_1920x1080(sigma)
    f, t = wl.frames[0], wl.templates[0]
    print(f"scene 1920x1080, 64x64 template, sigma {sigma}, tile-local form", flush=True)
    used, rho, deg, en = _run(S, ctx, f, t, sigma, S.SNCC_FORM_TILE_LOCAL)
    assert used == S.SNCC_FORM_TILE_LOCAL
    ta = O.precompute_template_approximation(t, sigma)
    want = pool.maps([(f, ta)])[0]
    err = _check(S, f, t, sigma, used, rho, deg, en, want=want)
    u, v, _ = O.argmax(want)
    if O.top2_margin(want) > 1e-4:
        assert np.unravel_index(np.argmax(rho), rho.shape) == (v, u)
    print(f"  max|drho| {err:.2e}", flush=True)


def test_texture_3840x2160_t128_tile_local(S, ctx, pool):
    wl = synth.texture_3840x2160(128)
    f, t = wl.frames[0], wl.templates[0]
    print("texture 3840x2160, 128x128 template, sigma 4, tile-local form", flush=True)
    used, rho, deg, en = _run(S, ctx, f, t, 4, S.SNCC_FORM_TILE_LOCAL)
    assert used == S.SNCC_FORM_TILE_LOCAL
    ta = O.precompute_template_approximation(t, 4)
    want = pool.maps([(f, ta)])[0]
    err = _check(S, f, t, 4, used, rho, deg, en, want=want)
    u, v, _ = O.argmax(want)
    assert O.top2_margin(want) > 1e-4
    assert np.unravel_index(np.argmax(rho), rho.shape) == (v, u)
    print(f"  K {ta.K}: max|drho| {err:.2e}", flush=True)
