"""The C ABI from several host threads without a GPU: the error message is
per thread (a call that fails in one thread leaves another thread's message
alone), and host-side validation gives each thread its own result while
other threads validate at the same time."""
import ctypes
import threading

from paper_1906_04576_amd import mr

# one invalid argument per thread, each named in its own message
BAD = [
    (3841, 2160, mr.MaskParams(), "divisible"),
    (64, 64, mr.MaskParams(level_enable=0b0111), "level_enable"),
    (64, 64, mr.MaskParams(sigma2=(-1.0, 1.848, 3.696, 0.0)), "sigma2"),
    (64, 64, mr.MaskParams(weight=(0.0, 50.0, 20.0, 1.0)), "weight"),
    (64, 64, mr.MaskParams(normal_cos=1.5), "normal_cos"),
    (0, 2160, mr.MaskParams(), "outside"),
]


def test_error_messages_are_per_thread():
    L = mr.lib()
    n = len(BAD)
    gate = threading.Barrier(n, timeout=60)
    got = [None] * n

    def work(k):
        W, H, mp, _ = BAD[k]
        cam, cmp = mr.mr_camera(W, H, 100.0), mp.c()
        msgs = []
        for _ in range(50):
            rc = L.mr_workspace_bytes(ctypes.byref(cam), ctypes.byref(cmp), mr.MR_EFFECT_SSAO)
            # every thread has failed once before any reads its message
            gate.wait()
            msgs.append((rc, L.mr_last_error().decode()))
            gate.wait()
        got[k] = msgs

    ts = [threading.Thread(target=work, args=(k,)) for k in range(n)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for k, msgs in enumerate(got):
        assert msgs is not None
        for rc, msg in msgs:
            assert rc == 0
            assert BAD[k][3] in msg, (k, msg)


def test_concurrent_validation_gives_every_thread_its_own_result():
    good = [(3840, 2160), (1920, 1080), (640, 360), (256, 256)]
    want = {wh: mr.mr_workspace_bytes(wh[0], wh[1], 1000.0, mr.MaskParams(), mr.MR_EFFECT_SSAO) for wh in good}
    errors = []

    def work(k):
        try:
            for i in range(200):
                wh = good[(k + i) % len(good)]
                assert mr.mr_workspace_bytes(wh[0], wh[1], 1000.0, mr.MaskParams(), mr.MR_EFFECT_SSAO) == want[wh]
                W, H, mp, key = BAD[(k + i) % len(BAD)]
                try:
                    mr.mr_workspace_bytes(W, H, 100.0, mp, mr.MR_EFFECT_SSAO)
                    errors.append((k, i, "accepted"))
                except mr.MRError as e:
                    if key not in str(e):
                        errors.append((k, i, str(e)))
        except Exception as e:  # a thread that raised must fail the test
            errors.append((k, repr(e)))

    ts = [threading.Thread(target=work, args=(k,)) for k in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors[:5]
