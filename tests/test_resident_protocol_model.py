"""Host-thread model of the LDS-resident variant's halo-swap protocol (the kernel in
``resident.hip``), run on the CPU: threads in the role of workgroups, numpy arrays in the role of
LDS tiles and of the two global exchange fields.  Each thread, per epoch of tb steps: publishes its
tile to the epoch's exchange field, raises its counter, waits (bounded) for its eight neighbours'
counters, reads its r*tb-deep halo ring from the exchange field, and advances its tile tb levels
on the shrinking region; at the end it writes its tile to `out`.  Exchange field of epoch e: the
workspace when (E - 1 - e) is even, else `out`.

Random delays between every step (and inside the halo reads) shuffle the interleavings; the
results must equal the plain definition (an FP64 Jacobi loop written here from the update rule),
so a workgroup that overwrote an exchange field a neighbour was still reading would show up as a
wrong cell.  A run in which one workgroup never publishes (a stalled tile) must end with every
thread out of its loop and the give-up recorded."""
import random
import threading
import time

import numpy as np
import pytest


def jacobi(u, W, b, steps):
    r = (W.shape[0] - 1) // 2
    x = u.astype(np.float64)
    for _ in range(steps):
        e = np.full((x.shape[0] + 2 * r, x.shape[1] + 2 * r), b)
        e[r:-r, r:-r] = x
        y = np.zeros_like(x)
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                y += W[dy + r, dx + r] * e[r + dy:r + dy + x.shape[0], r + dx:r + dx + x.shape[1]]
        x = y
    return x


def part(i, n, length):
    return (length * i) // n


def run_protocol(u0, W, b, steps, tb, gy, gx, seed, spin_limit=200000, stall=None):
    rows, cols = u0.shape
    r = (W.shape[0] - 1) // 2
    H = r * tb
    E = (steps + tb - 1) // tb
    ws = np.full((rows, cols), np.nan)
    out = np.full((rows, cols), np.nan)
    flags = [0] * (gy * gx)
    status = {"gave_up": 0, "rec": None}
    lock = threading.Lock()
    rng = random.Random(seed)
    delays = [rng.uniform(0, 2e-4) for _ in range(gy * gx)]

    def nap(w, scale=1.0):
        if random.random() < 0.5:
            time.sleep(delays[w] * scale)

    def wg(w):
        ty, tx = divmod(w, gx)
        y0, y1 = part(ty, gy, rows), part(ty + 1, gy, rows)
        x0, x1 = part(tx, gx, cols), part(tx + 1, gx, cols)
        th, tw = y1 - y0, x1 - x0
        tile = np.zeros((th + 2 * H, tw + 2 * H))
        tile[H:H + th, H:H + tw] = u0[y0:y1, x0:x1]
        for e in range(E):
            xg = ws if (E - 1 - e) % 2 == 0 else out
            if stall == w:
                return  # this workgroup never publishes: its neighbours must give up
            nap(w)
            xg[y0:y1, x0:x1] = tile[H:H + th, H:H + tw]
            nap(w)
            flags[w] = e + 1
            spins = 0
            quit_ = False
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ny, nx = ty + dy, tx + dx
                    if (dy, dx) == (0, 0) or not (0 <= ny < gy and 0 <= nx < gx):
                        continue
                    while flags[ny * gx + nx] < e + 1:
                        spins += 1
                        if spins % 64 == 0 and status["gave_up"]:
                            quit_ = True
                            break
                        if spins > spin_limit:
                            with lock:
                                if not status["gave_up"]:
                                    status["gave_up"] = 1
                                    status["rec"] = (w, e + 1, ny * gx + nx)
                            quit_ = True
                            break
                        time.sleep(0)
                    if quit_:
                        break
                if quit_:
                    break
            if quit_:
                return
            # the halo ring, read slowly cell by cell (a neighbour racing ahead would overwrite it)
            for y in range(th + 2 * H):
                for x in range(tw + 2 * H):
                    if H <= y < H + th and H <= x < H + tw:
                        continue
                    gyy, gxx = y0 + y - H, x0 + x - H
                    tile[y, x] = xg[gyy, gxx] if (0 <= gyy < rows and 0 <= gxx < cols) else b
                if y % 3 == 0:
                    nap(w, 0.2)
            levels = min(tb, steps - e * tb)
            for lev in range(1, levels + 1):
                lo = lev * r
                nxt = tile.copy()
                for y in range(lo, th + 2 * H - lo):
                    for x in range(lo, tw + 2 * H - lo):
                        gyy, gxx = y0 + y - H, x0 + x - H
                        if not (0 <= gyy < rows and 0 <= gxx < cols):
                            nxt[y, x] = b
                            continue
                        nxt[y, x] = float(np.sum(W * tile[y - r:y + r + 1, x - r:x + r + 1]))
                tile = nxt
        nap(w)
        out[y0:y1, x0:x1] = tile[H:H + th, H:H + tw]

    ths = [threading.Thread(target=wg, args=(w,)) for w in range(gy * gx)]
    for t in ths:
        t.start()
    for t in ths:
        t.join(timeout=300)
        assert not t.is_alive(), "a workgroup did not leave its loop"
    return out, status


@pytest.mark.parametrize("rows,cols,r,tb,steps,gy,gx", [(23, 29, 1, 3, 10, 3, 4), (20, 18, 2, 2, 7, 2, 3),
                                                       (16, 16, 1, 4, 4, 2, 2), (15, 40, 1, 2, 9, 3, 5)])
def test_resident_protocol_matches_the_definition(rows, cols, r, tb, steps, gy, gx):
    rng = np.random.default_rng(rows * cols + r)
    W = rng.random((2 * r + 1, 2 * r + 1))
    W /= W.sum()
    u0 = rng.random((rows, cols))
    ref = jacobi(u0, W, 0.5, steps)
    for seed in (1, 2):
        out, status = run_protocol(u0, W, 0.5, steps, tb, gy, gx, seed)
        assert status["gave_up"] == 0
        np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_resident_protocol_gives_up_and_ends():
    rng = np.random.default_rng(3)
    W = np.full((3, 3), 1.0 / 9)
    u0 = rng.random((18, 18))
    out, status = run_protocol(u0, W, 0.0, 9, 3, 3, 3, 4, spin_limit=500, stall=4)
    assert status["gave_up"] == 1
    w, want, nb = status["rec"]
    assert nb == 4 and want == 1  # a neighbour of the stalled centre gave up waiting for its first epoch
